// Second-order path and FP64 polish, on the stored FP64 operator in
// operator order.
//
// CG-Newton (section 2: pseudo-Huber function (7), smoothed problem (8),
// Newton model (9); section 8.1 item pdNCG and section 8.3 parameters):
// the Newton direction solves grad^2 f_mu(x) d = -grad f_mu(x) by
// preconditioned CG with the inverse Hessian diagonal as preconditioner,
// stopped at relative residual pcg_rtol; an Armijo backtracking line search
// of at most max_backtrack halvings sets the step.
//
// Polish: the reduced problem (13) of section 3.2 on the support S and signs
// of a given x, A_S^T A_S x_S = A_S^T b - tau sign_S, by preconditioned CG
// from x_S, followed by the optimality check of problem (1) (drop sign
// violators, add coordinates with |A_j^T (A x - b)| > tau), repeated.
//
// Both use one PCG whose Hessian-vector product is a CSR pass (t = A p) and
// a CSC pass with the epilogue Hp = mask (A^T t + d p) and the partial sums
// of p^T Hp; alpha and beta are formed on the device.
#include <algorithm>
#include <chrono>
#include <functional>
#include <cmath>
#include <cstring>

#include "common.hpp"
#include "kernels.hpp"

using namespace l1ls;

l1ls_status gap_fp64(const l1ls_instance* I, double tau, const double* x, double* P, double* D, double* gap,
                     hipStream_t s, DevAlloc* al = nullptr);
l1ls_status rel_err_planted(const l1ls_instance* I, const double* x, double* out, hipStream_t s);
void mf_apply_fwd(const l1ls_instance* I, const double* x, double* wn, double* out, hipStream_t s);
void mf_apply_adj(const l1ls_instance* I, const double* y, double* vm, double* out, hipStream_t s);
int64_t mf_wbuf_len(const l1ls_instance* I);
int64_t mf_vbuf_len(const l1ls_instance* I);
void mf_hess(const l1ls_instance* I, const double* p, double* wn, double* vm, const double* d, const uint8_t* mask,
             double* hp, double* part, const int32_t* done, hipStream_t s, bool f32);
int mf_grid(int64_t pairs);

namespace {

inline dim3 g1d(int64_t N) { return dim3((unsigned)std::max<int64_t>(1, (N + L1LS_BLOCK - 1) / L1LS_BLOCK)); }
inline int tgrid(int64_t N) { return (int)std::max<int64_t>(1, ((N + kTile - 1) / kTile + 3) / 4); }
constexpr int kRedBlocks = 512;   // grid of the vector kernels with partial sums

struct CgScalars {
    double rz, pHp, alpha, beta, rr, stop2;
    int32_t done;
    int32_t mnorm;  // 1: the stop test reads r^T M^-1 r (the preconditioned residual), 0: r^T r
};

// tile_products (kernels.hpp) with stored values of type TV widened to the
// FP64 of the vectors: val[k] * vec[idx[k]] for the tile's entries.
template <int NQ, typename TV>
__device__ __forceinline__ void tile_products_mixed(const int32_t* __restrict__ idx, const TV* __restrict__ val,
                                                    const double* __restrict__ vec, int32_t beg, int32_t cnt,
                                                    double* __restrict__ lds, int lane) {
    if (cnt <= 0) return;  // wave-uniform
    const int32_t* __restrict__ ib = idx + beg;
    const TV* __restrict__ vb = val + beg;
    const int32_t last = cnt - 1;
    int32_t c[NQ];
    TV v[NQ];
    double g[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) c[q] = __builtin_nontemporal_load(ib + min(q * kTile + lane, last));
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = __builtin_nontemporal_load(vb + min(q * kTile + lane, last));
#pragma unroll
    for (int q = 0; q < NQ; ++q) g[q] = ld_off32(vec, c[q]);
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds[q * kTile + lane] = (q * kTile + lane <= last) ? (double)v[q] * g[q] : 0.0;
    for (int32_t k = NQ * kTile + lane; k <= last; k += kTile) lds[k] = (double)vb[k] * ld_off32(vec, ib[k]);
}

// out = A in (CSR) or A^T in (CSC): one tile of 64 rows per wave.  TV: the
// stored values (FP64, or FP32 for the Hessian-vector products of the
// Newton directions); vectors and sums are FP64.  Skipped once the PCG the
// product belongs to has finished (cs->done).
template <typename TV>
__global__ __launch_bounds__(L1LS_BLOCK) void k_tile_spmv(const int32_t* __restrict__ ptr,
                                                          const int32_t* __restrict__ idx,
                                                          const TV* __restrict__ val,
                                                          const double* __restrict__ in, double* __restrict__ out,
                                                          int64_t rows, const CgScalars* __restrict__ cs) {
    if (cs && cs->done) return;
    __shared__ double lds[L1LS_BLOCK / L1LS_WAVE][kTile * kMaxNnz];
    const int lane = threadIdx.x % L1LS_WAVE, wid = threadIdx.x / L1LS_WAVE;
    const int64_t row0 = ((int64_t)blockIdx.x * (L1LS_BLOCK / L1LS_WAVE) + wid) * kTile;
    const int64_t i = row0 + lane;
    int32_t pb = 0, pe = 0;
    if (i < rows) {
        pb = ptr[i];
        pe = ptr[i + 1];
    }
    const int lastlane = (row0 + kTile <= rows) ? kTile - 1 : (rows > row0 ? (int)(rows - row0 - 1) : 0);
    const int32_t beg = __builtin_amdgcn_readfirstlane(__shfl(pb, 0, L1LS_WAVE));
    const int32_t end = __builtin_amdgcn_readfirstlane(__shfl(pe, lastlane, L1LS_WAVE));
    if (row0 < rows) tile_products_mixed<16, TV>(idx, val, in, beg, end - beg, lds[wid], lane);
    __syncthreads();
    if (i < rows) {
        double acc = 0.0;
        for (int32_t k = pb - beg; k < pe - beg; ++k) acc += lds[wid][k];
        out[i] = acc;
    }
}

// Hp = mask (A^T t + d p) over the CSC; part[block] = sum p Hp.
template <typename TV>
__global__ __launch_bounds__(L1LS_BLOCK) void k_hess(const int32_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ row,
                                                     const TV* __restrict__ val,
                                                     const double* __restrict__ t, const double* __restrict__ p,
                                                     const double* __restrict__ d, const uint8_t* __restrict__ mask,
                                                     double* __restrict__ hp, int64_t n, double* __restrict__ part,
                                                     const CgScalars* __restrict__ cs) {
    if (cs->done) return;
    __shared__ double lds[L1LS_BLOCK / L1LS_WAVE][kTile * kMaxNnz];
    const int lane = threadIdx.x % L1LS_WAVE, wid = threadIdx.x / L1LS_WAVE;
    const int64_t col0 = ((int64_t)blockIdx.x * (L1LS_BLOCK / L1LS_WAVE) + wid) * kTile;
    const int64_t j = col0 + lane;
    int32_t pb = 0, pe = 0;
    if (j < n) {
        pb = ptr[j];
        pe = ptr[j + 1];
    }
    const int lastlane = (col0 + kTile <= n) ? kTile - 1 : (n > col0 ? (int)(n - col0 - 1) : 0);
    const int32_t beg = __builtin_amdgcn_readfirstlane(__shfl(pb, 0, L1LS_WAVE));
    const int32_t end = __builtin_amdgcn_readfirstlane(__shfl(pe, lastlane, L1LS_WAVE));
    if (col0 < n) tile_products_mixed<16, TV>(row, val, t, beg, end - beg, lds[wid], lane);
    __syncthreads();
    double v[1] = {0.0};
    if (j < n) {
        double acc = 0.0;
        for (int32_t k = pb - beg; k < pe - beg; ++k) acc += lds[wid][k];
        const double pj = p[j];
        double h = acc + (d ? d[j] * pj : 0.0);
        if (mask && !mask[j]) h = 0.0;
        hp[j] = h;
        v[0] = pj * h;
    }
    block_reduce_stats<1, 1>(v);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// part[block] = (sum |x_j| over n, sum r_i^2 over m): the two terms of the
// objective f_tau(x) = tau ||x||_1 + 0.5 ||A x - b||^2 (problem (1)).
__global__ __launch_bounds__(L1LS_BLOCK) void k_obj_parts(const double* __restrict__ x, int64_t n,
                                                          const double* __restrict__ r, int64_t m,
                                                          double* __restrict__ part) {
    double v[2] = {0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) v[0] += fabs(x[j]);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) v[1] += r[i] * r[i];
    block_reduce_stats<2, 2>(v);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x + 0] = v[0];
        part[2 * blockIdx.x + 1] = v[1];
    }
}

// alpha = rz / p^T Hp  (one workgroup, fixed-order sum of the partials)
__global__ __launch_bounds__(1024) void k_cg_alpha(const double* __restrict__ part, int np, CgScalars* cs) {
    if (cs->done) return;
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < np; b += blockDim.x) v[0] += part[b];
    block_reduce_stats<1, 1>(v);
    if (threadIdx.x == 0) {
        cs->pHp = v[0];
        cs->alpha = (v[0] > 0.0) ? cs->rz / v[0] : 0.0;
        if (!(v[0] > 0.0)) cs->done = 1;  // no descent left (H p = 0) or breakdown
    }
}

// x += alpha p; r -= alpha Hp; z = minv r (masked); part = (r z, r r)
__global__ __launch_bounds__(L1LS_BLOCK) void k_cg_update(double* __restrict__ x, double* __restrict__ r,
                                                          double* __restrict__ z, const double* __restrict__ p,
                                                          const double* __restrict__ hp,
                                                          const double* __restrict__ minv,
                                                          const uint8_t* __restrict__ mask, int64_t n,
                                                          double* __restrict__ part, const CgScalars* __restrict__ cs) {
    if (cs->done) return;
    const double a = cs->alpha;
    double v[2] = {0.0, 0.0};
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        x[j] += a * p[j];
        const double rj = r[j] - a * hp[j];
        r[j] = rj;
        const double zj = (mask && !mask[j]) ? 0.0 : minv[j] * rj;
        z[j] = zj;
        v[0] += rj * zj;
        v[1] += rj * rj;
    }
    block_reduce_stats<2, 2>(v);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = v[0];
        part[2 * blockIdx.x + 1] = v[1];
    }
}

// beta = rz_new / rz; stop when ||r||^2 <= stop2
__global__ __launch_bounds__(1024) void k_cg_beta(const double* __restrict__ part, int np, CgScalars* cs,
                                                  int32_t* __restrict__ iters) {
    if (cs->done) return;
    double v[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < np; b += blockDim.x) {
        v[0] += part[2 * b];
        v[1] += part[2 * b + 1];
    }
    block_reduce_stats<2, 2>(v);
    if (threadIdx.x == 0) {
        cs->beta = (cs->rz != 0.0) ? v[0] / cs->rz : 0.0;
        cs->rz = v[0];
        cs->rr = v[1];
        *iters += 1;
        const double res2 = cs->mnorm ? v[0] : v[1];
        if (res2 <= cs->stop2 || !(res2 == res2)) cs->done = 1;
    }
}

// p = z + beta p
__global__ void k_cg_dir(double* __restrict__ p, const double* __restrict__ z, int64_t n,
                         const CgScalars* __restrict__ cs) {
    if (cs->done) return;
    const double be = cs->beta;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        p[j] = z[j] + be * p[j];
}

// Start of PCG: r = rhs - H x0 (hx given), z = minv r, p = z;
// part = (r z, r r, rhs rhs, rhs minv rhs)
__global__ __launch_bounds__(L1LS_BLOCK) void k_cg_start(const double* __restrict__ rhs,
                                                         const double* __restrict__ hx, double* __restrict__ r,
                                                         double* __restrict__ z, double* __restrict__ p,
                                                         const double* __restrict__ minv,
                                                         const uint8_t* __restrict__ mask, int64_t n,
                                                         double* __restrict__ part) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const bool on = !mask || mask[j];
        const double rj = on ? rhs[j] - (hx ? hx[j] : 0.0) : 0.0;
        const double zj = on ? minv[j] * rj : 0.0;
        r[j] = rj;
        z[j] = zj;
        p[j] = zj;
        v[0] += rj * zj;
        v[1] += rj * rj;
        v[2] += on ? rhs[j] * rhs[j] : 0.0;
        v[3] += on ? rhs[j] * (minv[j] * rhs[j]) : 0.0;
    }
    block_reduce_stats<4, 4>(v);
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x] = v[0];
        part[4 * blockIdx.x + 1] = v[1];
        part[4 * blockIdx.x + 2] = v[2];
        part[4 * blockIdx.x + 3] = v[3];
    }
}

// mnorm = 0: stop once ||r|| <= rtol ||rhs|| (the relative residual of the
// Newton systems); mnorm = 1: once r^T M^-1 r <= rtol^2 rhs^T M^-1 rhs, the
// residual of the diagonally scaled system, which bounds the error of every
// coordinate relative to its own scale however widely the diagonal of H
// spreads.
__global__ __launch_bounds__(1024) void k_cg_init(const double* __restrict__ part, int np, CgScalars* cs,
                                                  double rtol, int mnorm, int32_t* __restrict__ iters) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < np; b += blockDim.x) {
        v[0] += part[4 * b];
        v[1] += part[4 * b + 1];
        v[2] += part[4 * b + 2];
        v[3] += part[4 * b + 3];
    }
    block_reduce_stats<4, 4>(v);
    if (threadIdx.x == 0) {
        cs->rz = v[0];
        cs->rr = v[1];
        cs->mnorm = mnorm;
        cs->stop2 = rtol * rtol * (mnorm ? v[3] : v[2]);
        cs->alpha = cs->beta = cs->pHp = 0.0;
        cs->done = ((mnorm ? v[0] : v[1]) <= cs->stop2) ? 1 : 0;
        *iters = 0;
    }
}

__global__ void k_cg_reset(CgScalars* cs) {
    cs->rz = cs->pHp = cs->alpha = cs->beta = cs->rr = cs->stop2 = 0.0;
    cs->done = 0;
    cs->mnorm = 0;
}

// ---- CG-Newton vector kernels -------------------------------------------
// From g = A^T r (r = A x - b), form grad f_mu, the Hessian diagonal d,
// the preconditioner 1/(diag(A^T A) + d); part = (max |grad|, sum psi_mu(x)).
__global__ __launch_bounds__(L1LS_BLOCK) void k_newton_grad(const double* __restrict__ atr,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ gd,
                                                            const double* __restrict__ colnorm2, double tau,
                                                            double mu, int primal, double* __restrict__ grad,
                                                            double* __restrict__ d, double* __restrict__ minv,
                                                            int64_t n, double* __restrict__ part) {
    double v[2] = {0.0, 0.0};  // psi sum | max |grad|
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double xj = x[j];
        const double w = sqrt(mu * mu + xj * xj);
        const double gj = tau * xj / w + atr[j];
        const double dj = primal ? tau * mu * mu / (w * w * w) : tau * (1.0 - xj * gd[j] / w) / w;
        grad[j] = gj;
        d[j] = dj;
        minv[j] = 1.0 / (colnorm2[j] + dj);
        v[0] += w - mu;
        v[1] = fmax(v[1], fabs(gj));
    }
    block_reduce_stats<2, 1>(v);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = v[0];
        part[2 * blockIdx.x + 1] = v[1];
    }
}

// Duality-gap statistics of problem (1) at x from r = A x - b and
// g = A^T r: part = (sum r^2, sum b r, sum |x|, max |g|).
__global__ __launch_bounds__(L1LS_BLOCK) void k_gap_terms(const double* __restrict__ r,
                                                          const double* __restrict__ b,
                                                          const double* __restrict__ x,
                                                          const double* __restrict__ g, int64_t n, int64_t m,
                                                          double* __restrict__ part) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t N = n > m ? n : m;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < m) {
            v[0] += r[i] * r[i];
            v[1] += b[i] * r[i];
        }
        if (i < n) {
            v[2] += fabs(x[i]);
            v[3] = fmax(v[3], fabs(g[i]));
        }
    }
    block_reduce_stats<4, 3>(v);
    if (threadIdx.x == 0)
        for (int q = 0; q < 4; ++q) part[4 * blockIdx.x + q] = v[q];
}

// Power-method terms: part = (v . w, w . w).
__global__ __launch_bounds__(L1LS_BLOCK) void k_power_terms(const double* __restrict__ v,
                                                            const double* __restrict__ w, int64_t n,
                                                            double* __restrict__ part) {
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        acc[0] += v[i] * w[i];
        acc[1] += w[i] * w[i];
    }
    block_reduce_stats<2, 2>(acc);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = acc[0];
        part[2 * blockIdx.x + 1] = acc[1];
    }
}

// part = (grad . dx, sum psi_mu(x + a dx) | over m: sum (r + a q)^2)
__global__ __launch_bounds__(L1LS_BLOCK) void k_ls_terms(const double* __restrict__ x,
                                                         const double* __restrict__ dx,
                                                         const double* __restrict__ grad,
                                                         const double* __restrict__ r, const double* __restrict__ q,
                                                         double a, double mu, int64_t n, int64_t m,
                                                         double* __restrict__ part) {
    double v[3] = {0.0, 0.0, 0.0};
    const int64_t N = n > m ? n : m;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < n) {
            const double xn = x[i] + a * dx[i];
            v[0] += grad[i] * dx[i];
            v[1] += sqrt(mu * mu + xn * xn) - mu;
        }
        if (i < m) {
            const double ri = r[i] + a * q[i];
            v[2] += ri * ri;
        }
    }
    block_reduce_stats<3, 3>(v);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = v[0];
        part[3 * blockIdx.x + 1] = v[1];
        part[3 * blockIdx.x + 2] = v[2];
    }
}

// dual update of the primal-dual diagonal, then x += a dx
__global__ void k_newton_step(double* __restrict__ x, double* __restrict__ gd, const double* __restrict__ dx,
                              double a, double mu, int primal, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double xj = x[j];
    if (!primal) {
        const double w = sqrt(mu * mu + xj * xj);
        const double g0 = gd[j];
        const double g1 = g0 + (-g0 + xj / w + (1.0 - xj * g0 / w) * dx[j] / w);
        gd[j] = fmin(1.0, fmax(-1.0, g1));
    }
    x[j] = xj + a * dx[j];
}

// ---- polish kernels --------------------------------------------------------
// S = {j : |x_j| > thr}: mask and sign
__global__ void k_support_from_x(const double* __restrict__ x, uint8_t* __restrict__ mask,
                                 double* __restrict__ sgn, double thr, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double xj = x[j];
    const bool on = fabs(xj) > thr;
    mask[j] = on ? 1 : 0;
    sgn[j] = !on ? 0.0 : ((xj > 0.0) ? 1.0 : -1.0);
}

// rhs_j = (A^T b)_j - tau sgn_j on S; minv_j = 1 / diag(A^T A)_j
__global__ void k_polish_rhs(const double* __restrict__ atb, const double* __restrict__ sgn,
                             const uint8_t* __restrict__ mask, const double* __restrict__ colnorm2, double tau,
                             double* __restrict__ rhs, double* __restrict__ minv, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    rhs[j] = mask[j] ? atb[j] - tau * sgn[j] : 0.0;
    minv[j] = 1.0 / colnorm2[j];
}

// After a reduced solve: count (sign violators on S, KKT violators off S);
// violators change the mask/sign (drops first, adds only when none drop).
__global__ __launch_bounds__(L1LS_BLOCK) void k_polish_check(double* __restrict__ x, uint8_t* __restrict__ mask,
                                                             double* __restrict__ sgn, const double* __restrict__ atr,
                                                             double tau, double slack, int64_t n,
                                                             int32_t* __restrict__ counts) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (mask[j]) {
        const double xj = x[j];
        if (!(xj * sgn[j] > 0.0)) atomicAdd(counts + 0, 1);
    } else if (fabs(atr[j]) > tau * (1.0 + slack)) {
        atomicAdd(counts + 1, 1);
    }
}

__global__ void k_polish_apply(double* __restrict__ x, uint8_t* __restrict__ mask, double* __restrict__ sgn,
                               const double* __restrict__ atr, double tau, double slack, int drop, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (drop) {
        if (mask[j] && !(x[j] * sgn[j] > 0.0)) {
            mask[j] = 0;
            sgn[j] = 0.0;
            x[j] = 0.0;
        }
    } else if (!mask[j] && fabs(atr[j]) > tau * (1.0 + slack)) {
        mask[j] = 1;
        sgn[j] = (atr[j] > 0.0) ? -1.0 : 1.0;
    }
}

__global__ void k_mask_mul(double* __restrict__ x, const uint8_t* __restrict__ mask, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n && !mask[j]) x[j] = 0.0;
}

__global__ void k_fill_f64(double* __restrict__ out, double v, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) out[i] = v;
}

__global__ void k_axpby(const double* __restrict__ a, double alpha, const double* __restrict__ b, double beta,
                        double* __restrict__ out, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) out[i] = alpha * a[i] + beta * (b ? b[i] : 0.0);
}

// ---- block preconditioner of the polish ------------------------------------
// The reduced Hessian H_S = A_S^T A_S couples two columns of S only where they
// share a row, so it is block diagonal over the connected components of that
// relation: nearly all singletons, a few pairs and triples.  Two columns of a
// component can be nearly parallel (their largest sigma on the same Givens
// stencil), which the diagonal preconditioner leaves at condition numbers
// near kappa^2; with each small component's block inverted exactly the
// preconditioned system is the identity on S.

// Pairs (j, k), j < k, of masked columns that share row i, one thread per row.
__global__ __launch_bounds__(L1LS_BLOCK) void k_pairs_from_rows(const int32_t* __restrict__ ptr,
                                                                const int32_t* __restrict__ col,
                                                                const uint8_t* __restrict__ mask, int64_t m,
                                                                int32_t* __restrict__ pairs, int32_t cap,
                                                                int32_t* __restrict__ count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int32_t c[kMaxNnz];
    int k = 0;
    for (int32_t e = ptr[i]; e < ptr[i + 1] && k < kMaxNnz; ++e) {
        const int32_t j = col[e];
        if (mask[j]) c[k++] = j;
    }
    for (int a = 0; a < k; ++a)
        for (int b = a + 1; b < k; ++b) {
            const int32_t q = atomicAdd(count, 1);
            if (q < cap) {
                pairs[2 * q] = min(c[a], c[b]);
                pairs[2 * q + 1] = max(c[a], c[b]);
            }
        }
}

// Column cols[t] of the CSC (at most kMaxNnz entries) into slot t.
__global__ void k_pack_cols(const int32_t* __restrict__ ptr, const int32_t* __restrict__ row,
                            const double* __restrict__ val, const int32_t* __restrict__ cols, int32_t nc,
                            int32_t* __restrict__ prow, double* __restrict__ pval) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nc) return;
    const int32_t j = cols[t];
    const int32_t b = ptr[j], e = ptr[j + 1];
    for (int q = 0; q < kMaxNnz; ++q) {
        prow[(size_t)t * kMaxNnz + q] = (b + q < e) ? row[b + q] : -1;
        pval[(size_t)t * kMaxNnz + q] = (b + q < e) ? val[b + q] : 0.0;
    }
}

constexpr int kFixBlocks = 64;  // grid of k_block_fix (partial-sum slots after the kRedBlocks ones)

// z_j = sum_b W[t][b] v[bcol[t][b]] for member t (column mem[t]) of a block,
// replacing the diagonal z_j = minv_j v_j.  part slot (kRedBlocks + block) of
// stride `stride` receives sum v_j (z_j - minv_j v_j) at offset 0 and, when
// rhs is given, sum rhs_j ((M^-1 rhs)_j - minv_j rhs_j) at offset 3.  With
// p != nullptr, p_j = z_j as well (the PCG start).
__global__ __launch_bounds__(L1LS_BLOCK) void k_block_fix(const int32_t* __restrict__ mem,
                                                          const int32_t* __restrict__ boff,
                                                          const int32_t* __restrict__ bk,
                                                          const int32_t* __restrict__ bcol,
                                                          const double* __restrict__ w, int32_t nm,
                                                          const double* __restrict__ v, const double* __restrict__ minv,
                                                          double* __restrict__ z, double* __restrict__ p,
                                                          const double* __restrict__ rhs, double* __restrict__ part,
                                                          int stride, const CgScalars* __restrict__ cs) {
    if (cs && cs->done) return;
    double acc[2] = {0.0, 0.0};
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < nm; t += gridDim.x * blockDim.x) {
        const int32_t j = mem[t], o = boff[t], k = bk[t];
        double zn = 0.0, mr = 0.0;
        for (int b = 0; b < k; ++b) {
            const int32_t c = bcol[o + b];
            zn += w[(size_t)t * 16 + b] * v[c];
            if (rhs) mr += w[(size_t)t * 16 + b] * rhs[c];
        }
        acc[0] += v[j] * (zn - minv[j] * v[j]);
        if (rhs) acc[1] += rhs[j] * (mr - minv[j] * rhs[j]);
        z[j] = zn;
        if (p) p[j] = zn;
    }
    block_reduce_stats<2, 2>(acc);
    if (threadIdx.x == 0) {
        double* o = part + (size_t)stride * (kRedBlocks + blockIdx.x);
        for (int q = 0; q < stride; ++q) o[q] = 0.0;
        o[0] = acc[0];
        if (stride == 4) o[3] = acc[1];
    }
}

// ---- host side ------------------------------------------------------------
struct Work {
    const l1ls_instance* I = nullptr;
    hipStream_t s = nullptr;
    DevArena arena;
    double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *hp = nullptr, *minv = nullptr;
    double *d = nullptr, *rhs = nullptr, *tm = nullptr, *tm2 = nullptr, *grad = nullptr, *gd = nullptr;
    double* rres = nullptr;  // Newton residual A x - b (m); tm is PCG scratch
    double *xs = nullptr, *atr = nullptr, *atb = nullptr;
    double* part = nullptr;
    uint8_t* mask = nullptr;
    int32_t* counts = nullptr;
    int32_t* iters = nullptr;
    CgScalars* cs = nullptr;
    bool hv32 = false;  // Hessian-vector products of Newton directions with the FP32 values
    // Matrix-free operator (stage order, FP64): products from the rotation
    // tables, no stored A.  wn (n), vm (m) are its intermediate vectors.
    bool mf = false;
    double *wn = nullptr, *vm = nullptr;
    std::vector<double> h;
    // Block preconditioner of the polish (k_block_fix): nm members, their
    // columns, block offsets / sizes into bcol, and rows of the block inverses.
    int32_t nm = 0, mcap = 0;
    int32_t *bmem = nullptr, *boff = nullptr, *bk = nullptr, *bcol = nullptr, *pairs = nullptr, *npairs = nullptr;
    int32_t* prow = nullptr;
    double *bw = nullptr, *pval = nullptr;
    ~Work() {
        (void)hipStreamSynchronize(s);  // nothing queued may still use the buffers
        arena.release();
    }
    l1ls_status init(const l1ls_instance* inst, hipStream_t stream) {
        I = inst;
        s = stream;
        const int64_t n = I->n, m = I->m;
        for (double** v : {&x, &r, &z, &p, &hp, &minv, &d, &rhs, &grad, &gd, &xs, &atr, &atb})
            L1LS_TRY(arena.alloc(v, n));
        L1LS_TRY(arena.alloc(&tm, m));
        L1LS_TRY(arena.alloc(&tm2, m));
        L1LS_TRY(arena.alloc(&rres, m));
        L1LS_TRY(arena.alloc(&part, 4 * (size_t)std::max(kRedBlocks + kFixBlocks, tgrid(n))));
        L1LS_TRY(arena.alloc(&mask, n));
        L1LS_TRY(arena.alloc(&counts, 2));
        L1LS_TRY(arena.alloc(&iters, 1));
        L1LS_TRY(arena.alloc(&cs, 1));
        h.resize(4 * (size_t)std::max(kRedBlocks + kFixBlocks, tgrid(n)));
        return L1LS_OK;
    }
    // only what the products and a reduction need: x, atr (n), rres (m), part
    l1ls_status init_products(const l1ls_instance* inst, hipStream_t stream) {
        I = inst;
        s = stream;
        L1LS_TRY(arena.alloc(&x, I->n));
        L1LS_TRY(arena.alloc(&atr, I->n));
        L1LS_TRY(arena.alloc(&rres, I->m));
        L1LS_TRY(arena.alloc(&part, 4 * (size_t)std::max(kRedBlocks, tgrid(I->n))));
        h.resize(4 * (size_t)std::max(kRedBlocks, tgrid(I->n)));
        return L1LS_OK;
    }
    l1ls_status init_mf() {
        mf = true;
        L1LS_TRY(arena.alloc(&wn, mf_wbuf_len(I)));
        L1LS_TRY(arena.alloc(&vm, mf_vbuf_len(I)));
        return L1LS_OK;
    }
    // host sums of `k` statistics over `nb` partial slots (fixed order)
    l1ls_status host_sums(int k, int nb, double* out, bool max_last = false) {
        HIP_TRY(hipMemcpyAsync(h.data(), part, (size_t)k * nb * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int q = 0; q < k; ++q) out[q] = 0.0;
        for (int b = 0; b < nb; ++b)
            for (int q = 0; q < k; ++q) {
                const double v = h[(size_t)k * b + q];
                out[q] = (max_last && q == k - 1) ? std::max(out[q], v) : out[q] + v;
            }
        return L1LS_OK;
    }
    void spmv(const double* in, double* out) {  // out (m) = A in
        if (mf) {
            mf_apply_fwd(I, in, wn, out, s);
            return;
        }
        hipLaunchKernelGGL(k_tile_spmv<double>, dim3(tgrid(I->m)), dim3(L1LS_BLOCK), 0, s, I->csr_ptr, I->csr_col,
                           I->csr_v64, in, out, I->m, (const CgScalars*)nullptr);
    }
    void spmv_t(const double* in, double* out) {  // out (n) = A^T in
        if (mf) {
            mf_apply_adj(I, in, vm, out, s);
            return;
        }
        hipLaunchKernelGGL(k_tile_spmv<double>, dim3(tgrid(I->n)), dim3(L1LS_BLOCK), 0, s, I->csc_ptr, I->csc_row,
                           I->csc_v64, in, out, I->n, (const CgScalars*)nullptr);
    }
    // partial-sum slots written by hess()
    int hess_parts() const { return mf ? mf_grid(I->n / 2) : tgrid(I->n); }
    // H v = mask (A^T (A v) + dv v) into hp, inside a PCG (skipped once it is done)
    void hess(const double* v, const double* dv, const uint8_t* mk, bool f32) {
        const int64_t n = I->n;
        const int gt = tgrid(n);
        if (mf) {
            mf_hess(I, v, wn, vm, dv, mk, hp, part, &cs->done, s, f32);
            return;
        }
        if (f32) {
            hipLaunchKernelGGL(k_tile_spmv<float>, dim3(tgrid(I->m)), dim3(L1LS_BLOCK), 0, s, I->csr_ptr,
                               I->csr_col, I->csr_v32, v, tm, I->m, (const CgScalars*)cs);
            hipLaunchKernelGGL(k_hess<float>, dim3(gt), dim3(L1LS_BLOCK), 0, s, I->csc_ptr, I->csc_row, I->csc_v32,
                               tm, v, dv, mk, hp, n, part, (const CgScalars*)cs);
        } else {
            hipLaunchKernelGGL(k_tile_spmv<double>, dim3(tgrid(I->m)), dim3(L1LS_BLOCK), 0, s, I->csr_ptr,
                               I->csr_col, I->csr_v64, v, tm, I->m, (const CgScalars*)cs);
            hipLaunchKernelGGL(k_hess<double>, dim3(gt), dim3(L1LS_BLOCK), 0, s, I->csc_ptr, I->csc_row,
                               I->csc_v64, tm, v, dv, mk, hp, n, part, (const CgScalars*)cs);
        }
    }
    // Components of the masked columns that share rows (polish, stored FP64
    // operator): the exact inverse of each component's block of A_S^T A_S
    // (components of 2 to 16 columns; larger ones keep the diagonal).  The
    // result does not depend on the order in which pairs are found.
    l1ls_status setup_blocks() {
        nm = 0;
        constexpr int32_t kPairCap = 1 << 21;
        constexpr int kMaxBlk = 16;
        if (!pairs) {
            L1LS_TRY(arena.alloc(&pairs, 2 * (size_t)kPairCap));
            L1LS_TRY(arena.alloc(&npairs, 1));
        }
        HIP_TRY(hipMemsetAsync(npairs, 0, sizeof(int32_t), s));
        hipLaunchKernelGGL(k_pairs_from_rows, g1d(I->m), dim3(L1LS_BLOCK), 0, s, I->csr_ptr, I->csr_col, mask, I->m,
                           pairs, kPairCap, npairs);
        int32_t np = 0;
        HIP_TRY(hipMemcpyAsync(&np, npairs, sizeof(np), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (np <= 0 || np > kPairCap) return L1LS_OK;  // none, or too many to list: the diagonal alone
        std::vector<int32_t> hp2(2 * (size_t)np);
        HIP_TRY(hipMemcpy(hp2.data(), pairs, hp2.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        std::vector<uint64_t> keys(np);
        for (int32_t q = 0; q < np; ++q)
            keys[q] = ((uint64_t)(uint32_t)hp2[2 * q] << 32) | (uint32_t)hp2[2 * q + 1];
        std::sort(keys.begin(), keys.end());
        keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
        // union-find over the columns that appear in a pair
        std::vector<int32_t> cols;
        cols.reserve(2 * keys.size());
        for (uint64_t k : keys) {
            cols.push_back((int32_t)(k >> 32));
            cols.push_back((int32_t)(k & 0xffffffffu));
        }
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        auto id = [&](int32_t c) { return (int32_t)(std::lower_bound(cols.begin(), cols.end(), c) - cols.begin()); };
        std::vector<int32_t> par(cols.size());
        for (size_t q = 0; q < par.size(); ++q) par[q] = (int32_t)q;
        std::function<int32_t(int32_t)> root = [&](int32_t a) {
            while (par[a] != a) a = par[a] = par[par[a]];
            return a;
        };
        for (uint64_t k : keys) {
            int32_t a = root(id((int32_t)(k >> 32))), b = root(id((int32_t)(k & 0xffffffffu)));
            if (a != b) par[std::max(a, b)] = std::min(a, b);
        }
        // components in order of their smallest column; members ascending
        std::vector<std::vector<int32_t>> comp;
        std::vector<int32_t> cidx(cols.size(), -1);
        for (size_t q = 0; q < cols.size(); ++q) {
            const int32_t r0 = root((int32_t)q);
            if (cidx[r0] < 0) {
                cidx[r0] = (int32_t)comp.size();
                comp.emplace_back();
            }
            comp[cidx[r0]].push_back(cols[q]);
        }
        std::vector<int32_t> mcol, moff, mk, mbcol;
        for (auto& c : comp) {
            if (c.size() < 2 || c.size() > (size_t)kMaxBlk) continue;
            const int32_t off = (int32_t)mbcol.size();
            for (int32_t j : c) {
                mcol.push_back(j);
                moff.push_back(off);
                mk.push_back((int32_t)c.size());
            }
            mbcol.insert(mbcol.end(), c.begin(), c.end());
        }
        const int32_t nmem = (int32_t)mcol.size();
        if (nmem == 0) return L1LS_OK;
        if (nmem > mcap) {
            mcap = std::max(nmem, 4096);
            L1LS_TRY(arena.alloc(&bmem, mcap));
            L1LS_TRY(arena.alloc(&boff, mcap));
            L1LS_TRY(arena.alloc(&bk, mcap));
            L1LS_TRY(arena.alloc(&bcol, mcap));
            L1LS_TRY(arena.alloc(&bw, (size_t)16 * mcap));
            L1LS_TRY(arena.alloc(&prow, (size_t)kMaxNnz * mcap));
            L1LS_TRY(arena.alloc(&pval, (size_t)kMaxNnz * mcap));
        }
        // the members' columns of A (rows and FP64 values), to the host
        HIP_TRY(hipMemcpyAsync(bcol, mbcol.data(), nmem * sizeof(int32_t), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_pack_cols, dim3((nmem + 255) / 256), dim3(256), 0, s, I->csc_ptr, I->csc_row,
                           I->csc_v64, bcol, nmem, prow, pval);
        std::vector<int32_t> hrow((size_t)kMaxNnz * nmem);
        std::vector<double> hval((size_t)kMaxNnz * nmem);
        HIP_TRY(hipMemcpyAsync(hrow.data(), prow, hrow.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hval.data(), pval, hval.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        // per component: H_C = A_C^T A_C and its inverse (Gauss-Jordan with
        // partial pivoting); a numerically singular block keeps the diagonal
        std::vector<double> wrow((size_t)16 * nmem, 0.0);
        std::vector<uint8_t> keep(nmem, 1);
        for (int32_t t0 = 0; t0 < nmem;) {
            const int k = mk[t0];
            double H[kMaxBlk][2 * kMaxBlk];
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) {
                    double acc = 0.0;
                    const int32_t* ra = &hrow[(size_t)(t0 + a) * kMaxNnz];
                    const int32_t* rb = &hrow[(size_t)(t0 + b) * kMaxNnz];
                    for (int qa = 0; qa < kMaxNnz && ra[qa] >= 0; ++qa)
                        for (int qb = 0; qb < kMaxNnz && rb[qb] >= 0; ++qb)
                            if (ra[qa] == rb[qb])
                                acc += hval[(size_t)(t0 + a) * kMaxNnz + qa] * hval[(size_t)(t0 + b) * kMaxNnz + qb];
                    H[a][b] = acc;
                    H[a][k + b] = (a == b) ? 1.0 : 0.0;
                }
            bool ok = true;
            for (int c = 0; c < k && ok; ++c) {
                int piv = c;
                for (int a = c + 1; a < k; ++a)
                    if (std::fabs(H[a][c]) > std::fabs(H[piv][c])) piv = a;
                if (!(std::fabs(H[piv][c]) > 0.0)) {
                    ok = false;
                    break;
                }
                if (piv != c)
                    for (int b = 0; b < 2 * k; ++b) std::swap(H[c][b], H[piv][b]);
                const double inv = 1.0 / H[c][c];
                for (int b = 0; b < 2 * k; ++b) H[c][b] *= inv;
                for (int a = 0; a < k; ++a) {
                    if (a == c) continue;
                    const double f = H[a][c];
                    if (f != 0.0)
                        for (int b = 0; b < 2 * k; ++b) H[a][b] -= f * H[c][b];
                }
            }
            for (int a = 0; a < k; ++a) {
                if (!ok) keep[t0 + a] = 0;
                for (int b = 0; b < k; ++b) wrow[(size_t)(t0 + a) * 16 + b] = ok ? H[a][k + b] : 0.0;
            }
            t0 += k;
        }
        // drop the members of blocks that could not be inverted
        std::vector<int32_t> fcol, foff, fk;
        std::vector<double> fw;
        for (int32_t t = 0; t < nmem; ++t) {
            if (!keep[t]) continue;
            fcol.push_back(mcol[t]);
            foff.push_back(moff[t]);
            fk.push_back(mk[t]);
            fw.insert(fw.end(), wrow.begin() + (size_t)t * 16, wrow.begin() + (size_t)(t + 1) * 16);
        }
        nm = (int32_t)fcol.size();
        if (nm == 0) return L1LS_OK;
        HIP_TRY(hipMemcpyAsync(bmem, fcol.data(), nm * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(boff, foff.data(), nm * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(bk, fk.data(), nm * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(bw, fw.data(), fw.size() * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));  // the host vectors go out of scope
        return L1LS_OK;
    }
    // PCG on H v = rhs from v = x (in place), H = mask (A^T A + diag(dv)) mask.
    // zero_start: v is known to be 0, so H v = 0 is not computed.
    // f32: the products with A use its FP32 values (the Newton directions);
    // the polish keeps FP64.
    l1ls_status pcg(double* v, const double* rhs_v, const double* dv, const uint8_t* mk, double rtol, int maxit,
                    int* out_iters, bool zero_start = false, bool f32 = false, int mnorm = 0, bool blocks = false) {
        blocks = blocks && nm > 0;
        const int64_t n = I->n;
        const int gt = hess_parts();
        hipLaunchKernelGGL(k_cg_reset, dim3(1), dim3(1), 0, s, cs);
        if (!zero_start) hess(v, dv, mk, f32);  // H v for the starting residual
        hipLaunchKernelGGL(k_cg_start, dim3(kRedBlocks), dim3(L1LS_BLOCK), 0, s, rhs_v,
                           zero_start ? (const double*)nullptr : hp, r, z, p, minv, mk, n, part);
        // with blocks, their members' z (and p) and the two sums that read z
        const int np = blocks ? kRedBlocks + kFixBlocks : kRedBlocks;
        if (blocks)
            hipLaunchKernelGGL(k_block_fix, dim3(kFixBlocks), dim3(L1LS_BLOCK), 0, s, bmem, boff, bk, bcol, bw, nm, r,
                               minv, z, p, rhs_v, part, 4, (const CgScalars*)nullptr);
        hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(1024), 0, s, part, np, cs, rtol, mnorm, iters);
        HIP_TRY(hipGetLastError());
        const int batch = 8;
        int done_iters = 0;
        for (int it = 0; it < maxit; it += batch) {
            const int nb = std::min(batch, maxit - it);
            for (int q = 0; q < nb; ++q) {
                hess(p, dv, mk, f32);
                hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(1024), 0, s, part, gt, cs);
                hipLaunchKernelGGL(k_cg_update, dim3(kRedBlocks), dim3(L1LS_BLOCK), 0, s, v, r, z, p, hp, minv, mk,
                                   n, part, (const CgScalars*)cs);
                if (blocks)
                    hipLaunchKernelGGL(k_block_fix, dim3(kFixBlocks), dim3(L1LS_BLOCK), 0, s, bmem, boff, bk, bcol,
                                       bw, nm, r, minv, z, (double*)nullptr, (const double*)nullptr, part, 2,
                                       (const CgScalars*)cs);
                hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(1024), 0, s, part, np, cs, iters);
                hipLaunchKernelGGL(k_cg_dir, dim3(kRedBlocks), dim3(L1LS_BLOCK), 0, s, p, z, n,
                                   (const CgScalars*)cs);
            }
            HIP_TRY(hipGetLastError());
            CgScalars c;
            HIP_TRY(hipMemcpyAsync(&c, cs, sizeof(c), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(&done_iters, iters, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (c.done) break;
        }
        *out_iters = done_iters;
        return L1LS_OK;
    }
};

}  // namespace

// FP64 polish of x_dev (original order, n entries), in place; the starting
// support is {j : |x_j| > support_tol}.  x_dev keeps its value when the
// polished point's objective f_tau is larger.
l1ls_status polish_fp64(const l1ls_instance* I, double tau, double* x_dev, hipStream_t s, int* rounds_out,
                        int64_t* pcg_iters_out, double support_tol, DevAlloc* al = nullptr) {
    *rounds_out = 0;
    *pcg_iters_out = 0;
    if (!I->csr_v64 || !I->csc_v64) return L1LS_E_UNSUPPORTED;
    Work W;
    W.arena.al = al;
    L1LS_TRY(W.init(I, s));
    const int64_t n = I->n;
    hipLaunchKernelGGL((k_gather_perm<double, double>), g1d(n), dim3(L1LS_BLOCK), 0, s, x_dev, W.x, I->op_col_of, n);
    // f_tau at the starting point (the polish keeps it when it does not improve)
    auto objective = [&](const double* xv, double* f) -> l1ls_status {
        W.spmv(xv, W.tm);
        hipLaunchKernelGGL(k_axpby, g1d(I->m), dim3(L1LS_BLOCK), 0, s, W.tm, 1.0, I->b_op, -1.0, W.tm, I->m);
        hipLaunchKernelGGL(k_obj_parts, dim3(kRedBlocks), dim3(L1LS_BLOCK), 0, s, xv, n, (const double*)W.tm, I->m,
                           W.part);
        double sums[2];
        L1LS_TRY(W.host_sums(2, kRedBlocks, sums));
        *f = tau * sums[0] + 0.5 * sums[1];
        return L1LS_OK;
    };
    double f_in = 0.0;
    HIP_TRY(hipMemcpyAsync(W.grad, W.x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    L1LS_TRY(objective(W.x, &f_in));
    hipLaunchKernelGGL(k_support_from_x, g1d(n), dim3(L1LS_BLOCK), 0, s, W.x, W.mask, W.xs, support_tol, n);
    W.spmv_t(I->b_op, W.atb);
    const double slack = 1e-10;
    int64_t total = 0;
    int rounds = 0;
    for (rounds = 1; rounds <= 10; ++rounds) {
        hipLaunchKernelGGL(k_polish_rhs, g1d(n), dim3(L1LS_BLOCK), 0, s, W.atb, W.xs, W.mask, I->colnorm2_op, tau,
                           W.rhs, W.minv, n);
        hipLaunchKernelGGL(k_mask_mul, g1d(n), dim3(L1LS_BLOCK), 0, s, W.x, W.mask, n);
        int it = 0;
        // stop on the residual of the diagonally scaled system: column norms
        // of A_S spread over kappa^2, and a plain relative residual leaves
        // the coordinates of the smallest columns unresolved
        L1LS_TRY(W.setup_blocks());
        L1LS_TRY(W.pcg(W.x, W.rhs, nullptr, W.mask, 1e-13, 2000, &it, false, false, 1, true));
        total += it;
        // A^T (A x - b)
        W.spmv(W.x, W.tm);
        hipLaunchKernelGGL(k_axpby, g1d(I->m), dim3(L1LS_BLOCK), 0, s, W.tm, 1.0, I->b_op, -1.0, W.tm, I->m);
        W.spmv_t(W.tm, W.atr);
        HIP_TRY(hipMemsetAsync(W.counts, 0, 2 * sizeof(int32_t), s));
        hipLaunchKernelGGL(k_polish_check, g1d(n), dim3(L1LS_BLOCK), 0, s, W.x, W.mask, W.xs, W.atr, tau, slack, n,
                           W.counts);
        int32_t cnt[2];
        HIP_TRY(hipMemcpyAsync(cnt, W.counts, sizeof(cnt), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (std::getenv("L1LS_DEBUG_POLISH"))
            std::fprintf(stderr,
                         "l1ls polish: round %d, %d columns in blocks, %d PCG iterations, %d sign changes on S, "
                         "%d KKT violators off S\n",
                         rounds, W.nm, it, cnt[0], cnt[1]);
        if (cnt[0] == 0 && cnt[1] == 0) break;
        hipLaunchKernelGGL(k_polish_apply, g1d(n), dim3(L1LS_BLOCK), 0, s, W.x, W.mask, W.xs, W.atr, tau, slack,
                           cnt[0] > 0 ? 1 : 0, n);
    }
    // a polish that ends above the starting objective (a support still far
    // from the solution's after the last round) returns the starting point.
    // The comparison allows 1e-12 relative: both values carry FP64 rounding
    // of sums over the m + n terms of f_tau (up to a few units in 1e-15 were
    // seen between an iterate and its certified polish), and a polish from a
    // wrong support raises f_tau by far more.
    double f_out = 0.0;
    L1LS_TRY(objective(W.x, &f_out));
    const bool keep = f_out <= f_in + 1e-12 * fabs(f_in);
    if (std::getenv("L1LS_DEBUG_POLISH"))
        std::fprintf(stderr, "l1ls polish: f_tau %.17g -> %.17g (%s)\n", f_in, f_out, keep ? "kept" : "reverted");
    hipLaunchKernelGGL((k_gather_perm<double, double>), g1d(n), dim3(L1LS_BLOCK), 0, s, keep ? W.x : W.grad, x_dev,
                       I->op_col_pos, n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    *rounds_out = std::min(rounds, 10);
    *pcg_iters_out = total;
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_solve_cg_newton(const l1ls_instance* I, const l1ls_solve_opts* o, double* x_out,
                                            l1ls_report* rep) {
    if (!I || !o || !x_out) return L1LS_E_ARG;
    if (o->op != L1LS_OP_STORED && o->op != L1LS_OP_MATRIX_FREE) return L1LS_E_ARG;
    const bool mf = (o->op == L1LS_OP_MATRIX_FREE);
    // the matrix-free products are FP64 and work in stage order (the order
    // of the solver's vectors under the STAGE layout); the polish needs the
    // stored FP64 A
    if (mf && (!I->mf_emb || I->layout != L1LS_LAYOUT_STAGE ||
               I->m * (int64_t)sizeof(double) >= ((int64_t)1 << 32) ||
               (o->polish && (!I->csr_v64 || !I->csc_v64))))
        return L1LS_E_UNSUPPORTED;
    if (!mf && (!I->csr_v64 || !I->csc_v64)) return L1LS_E_UNSUPPORTED;
    if (o->max_iter < 0) return L1LS_E_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)o->stream;
    const double tau = o->tau > 0 ? o->tau : I->tau;
    const double mu = o->mu > 0 ? o->mu : 1e-5;
    const double prtol = o->pcg_rtol > 0 ? o->pcg_rtol : 0.1;
    const int maxbt = o->max_backtrack > 0 ? o->max_backtrack : 50;
    const int pcgmax = o->pcg_maxit > 0 ? o->pcg_maxit : 1000;
    const int primal = o->hessian == 1 ? 1 : 0;
    const double gtol = (o->rel_gap_tol > 0 ? o->rel_gap_tol : 1e-9) * tau;
    if (!is_finite(tau) || !is_finite(mu)) return L1LS_E_ARG;
    const int64_t n = I->n, m = I->m;
    Work W;
    W.hv32 = (o->precision == L1LS_F32);
    if (W.hv32 && !mf && (!I->csr_v32 || !I->csc_v32)) return L1LS_E_UNSUPPORTED;
    L1LS_TRY(W.init(I, s));
    if (mf) L1LS_TRY(W.init_mf());
    if (o->x0_dev)
        hipLaunchKernelGGL((k_gather_perm<double, double>), g1d(n), dim3(L1LS_BLOCK), 0, s, o->x0_dev, W.x,
                           I->op_col_of, n);
    else
        HIP_TRY(hipMemsetAsync(W.x, 0, n * sizeof(double), s));
    HIP_TRY(hipMemsetAsync(W.gd, 0, n * sizeof(double), s));
    int64_t newton = 0, pcg_total = 0;
    double gnorm = INFINITY;
    const double armijo = 1e-4;
    for (newton = 0; newton < o->max_iter; ++newton) {
        // r = A x - b; grad, diagonal, preconditioner
        W.spmv(W.x, W.rres);
        hipLaunchKernelGGL(k_axpby, g1d(m), dim3(L1LS_BLOCK), 0, s, W.rres, 1.0, I->b_op, -1.0, W.rres, m);
        W.spmv_t(W.rres, W.atr);
        hipLaunchKernelGGL(k_newton_grad, dim3(kRedBlocks), dim3(L1LS_BLOCK), 0, s, W.atr, W.x, W.gd,
                           I->colnorm2_op, tau, mu, primal, W.grad, W.d, W.minv, n, W.part);
        double gs[2];
        L1LS_TRY(W.host_sums(2, kRedBlocks, gs, true));
        gnorm = gs[1];
        if (!is_finite(gnorm)) return L1LS_E_NONFINITE;
        if (gnorm <= gtol) break;
        // Newton direction: H dx = -grad, from dx = 0
        hipLaunchKernelGGL(k_axpby, g1d(n), dim3(L1LS_BLOCK), 0, s, W.grad, -1.0, (const double*)nullptr, 0.0,
                           W.rhs, n);
        HIP_TRY(hipMemsetAsync(W.xs, 0, n * sizeof(double), s));
        int it = 0;
        L1LS_TRY(W.pcg(W.xs, W.rhs, W.d, nullptr, prtol, pcgmax, &it, true, W.hv32));
        pcg_total += it;
        // line search on f_mu(x + a dx) = tau sum psi + 0.5 ||r + a A dx||^2
        W.spmv(W.xs, W.tm2);
        double t0s[3];
        hipLaunchKernelGGL(k_ls_terms, dim3(kRedBlocks), dim3(L1LS_BLOCK), 0, s, W.x, W.xs, W.grad, W.rres, W.tm2,
                           0.0, mu, n, m, W.part);
        L1LS_TRY(W.host_sums(3, kRedBlocks, t0s));
        const double f0 = tau * t0s[1] + 0.5 * t0s[2];
        const double slope = t0s[0];
        double a = 1.0;
        for (int bt = 0; bt < maxbt; ++bt) {
            double ta[3];
            hipLaunchKernelGGL(k_ls_terms, dim3(kRedBlocks), dim3(L1LS_BLOCK), 0, s, W.x, W.xs, W.grad, W.rres,
                               W.tm2, a, mu, n, m, W.part);
            L1LS_TRY(W.host_sums(3, kRedBlocks, ta));
            if (tau * ta[1] + 0.5 * ta[2] <= f0 + armijo * a * slope) break;
            if (bt + 1 < maxbt) a *= 0.5;
        }
        hipLaunchKernelGGL(k_newton_step, g1d(n), dim3(L1LS_BLOCK), 0, s, W.x, W.gd, W.xs, a, mu, primal, n);
        HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL((k_gather_perm<double, double>), g1d(n), dim3(L1LS_BLOCK), 0, s, W.x, x_out, I->op_col_pos,
                       n);
    HIP_TRY(hipStreamSynchronize(s));
    l1ls_report r;
    std::memset(&r, 0, sizeof(r));
    r.iterations = newton;
    r.inner = pcg_total;
    int prounds = 0;
    int64_t ppcg = 0;
    if (o->polish) {
        // smoothed iterates carry |x_j| <~ 2 mu off the support (|x/w| < 1)
        L1LS_TRY(polish_fp64(I, tau, x_out, s, &prounds, &ppcg, 10.0 * mu));
        r.inner += ppcg;
    }
    r.polish_rounds = prounds;
    if (mf && !o->polish) {
        // FP64 certificate through the matrix-free products (stage order):
        // P = tau ||x||_1 + 0.5 ||r||^2, theta = min(1, tau / ||A^T r||_inf),
        // D = -0.5 theta^2 ||r||^2 - theta b^T r
        W.spmv(W.x, W.rres);
        hipLaunchKernelGGL(k_axpby, g1d(m), dim3(L1LS_BLOCK), 0, s, W.rres, 1.0, I->b_op, -1.0, W.rres, m);
        W.spmv_t(W.rres, W.atr);
        hipLaunchKernelGGL(k_gap_terms, dim3(kRedBlocks), dim3(L1LS_BLOCK), 0, s, W.rres, I->b_op, W.x, W.atr, n, m,
                           W.part);
        double gt4[4];
        L1LS_TRY(W.host_sums(4, kRedBlocks, gt4, true));
        const double theta = (gt4[3] <= tau) ? 1.0 : tau / gt4[3];
        r.primal = tau * gt4[2] + 0.5 * gt4[0];
        r.dual = -0.5 * theta * theta * gt4[0] - theta * gt4[1];
        r.rel_gap = (r.primal - r.dual) / std::fabs(r.primal);
        if (!is_finite(r.primal) || !is_finite(r.dual)) return L1LS_E_NONFINITE;
    } else {
        L1LS_TRY(gap_fp64(I, tau, x_out, &r.primal, &r.dual, &r.rel_gap, s));
    }
    L1LS_TRY(rel_err_planted(I, x_out, &r.rel_err, s));
    r.converged = (gnorm <= gtol) ? 1 : 0;
    r.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = r;
    return r.converged ? L1LS_OK : L1LS_NOT_CONVERGED;
}

// lambda_max(A^T A) by the power method (the FP64 estimate of L for sigma
// laws without a closed form): v_0 = v0 / ||v0|| (or the normalised all-ones
// vector), then per step w = A^T (A v), lambda = v . w, v = w / ||w||.
// Returns the last lambda.
extern "C" l1ls_status l1ls_power_iteration(const l1ls_instance* I, int32_t op, int32_t iters, const double* v0_dev,
                                            double* lambda_out, void* stream) {
    if (!I || !lambda_out || iters < 1) return L1LS_E_ARG;
    if (op != L1LS_OP_STORED && op != L1LS_OP_MATRIX_FREE) return L1LS_E_ARG;
    const bool mf = (op == L1LS_OP_MATRIX_FREE);
    if (!mf && (!I->csr_v64 || !I->csc_v64)) return L1LS_E_UNSUPPORTED;
    if (mf && (!I->mf_emb || I->layout != L1LS_LAYOUT_STAGE || I->m * (int64_t)sizeof(double) >= ((int64_t)1 << 32)))
        return L1LS_E_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = I->n;
    Work W;
    L1LS_TRY(W.init_products(I, s));
    if (mf) L1LS_TRY(W.init_mf());
    // v in operator order (W.x), w = A^T A v (W.atr), A v in W.rres
    if (v0_dev)
        hipLaunchKernelGGL((k_gather_perm<double, double>), g1d(n), dim3(L1LS_BLOCK), 0, s, v0_dev, W.x,
                           I->op_col_of, n);
    else
        hipLaunchKernelGGL(k_fill_f64, g1d(n), dim3(L1LS_BLOCK), 0, s, W.x, 1.0, n);
    double t2[2];
    hipLaunchKernelGGL(k_power_terms, dim3(kRedBlocks), dim3(L1LS_BLOCK), 0, s, W.x, W.x, n, W.part);
    L1LS_TRY(W.host_sums(2, kRedBlocks, t2));
    if (!(t2[1] > 0.0) || !is_finite(t2[1])) return L1LS_E_ARG;
    hipLaunchKernelGGL(k_axpby, g1d(n), dim3(L1LS_BLOCK), 0, s, W.x, 1.0 / std::sqrt(t2[1]),
                       (const double*)nullptr, 0.0, W.x, n);
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        W.spmv(W.x, W.rres);
        W.spmv_t(W.rres, W.atr);
        hipLaunchKernelGGL(k_power_terms, dim3(kRedBlocks), dim3(L1LS_BLOCK), 0, s, W.x, W.atr, n, W.part);
        L1LS_TRY(W.host_sums(2, kRedBlocks, t2));
        lam = t2[0];
        if (!is_finite(lam) || !is_finite(t2[1])) return L1LS_E_NONFINITE;
        if (!(t2[1] > 0.0)) break;  // A v = 0: v is in the null space (lambda = 0)
        hipLaunchKernelGGL(k_axpby, g1d(n), dim3(L1LS_BLOCK), 0, s, W.atr, 1.0 / std::sqrt(t2[1]),
                           (const double*)nullptr, 0.0, W.x, n);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    *lambda_out = lam;
    return L1LS_OK;
}
