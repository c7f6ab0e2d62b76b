// Streaming kernels of the FISTA hot path (section 8.1, FISTA on problem
// (1)) over the stored operator:
//   residual pass  (CSR):  r_x = A x_k - b,  r_y = (1+beta_k) r_x - beta_k r_x,prev
//   transpose pass (CSC):  g = A^T r_y,  y = x_{k-1} + beta (x_{k-1} - x_{k-2}),
//                          x_k = soft(y - g/L, tau/L)
// plus FP64 partial statistics for the duality gap.  Each row (column) is
// handled by a segment of W lanes of a wave64; a grid-stride loop keeps the
// grid fixed so the partial arrays have one slot per workgroup and every
// reduction runs in a fixed order (bitwise reproducible).
#pragma once

#include "common.hpp"

namespace l1ls {

struct GapState {
    double P, D, gap;
    double ginf, l1, rr;
    int64_t iter;       // iteration of the last evaluated gap
    int64_t conv_iter;  // iteration at which the test passed (-1: not yet)
    int32_t done;       // 1 once converged (or non-finite): later passes are no-ops
    int32_t nonfinite;
};

// sign(z) max(|z| - thr, 0); a NaN z stays NaN so that the gap test sees it.
template <typename T>
__device__ __forceinline__ T soft_threshold(T z, T thr) {
    const T az = fabs(z);
    return (az <= thr) ? T(0) : copysign(az - thr, z);
}

constexpr int kTile = 64;      // rows (columns) per wave
constexpr int kMaxNnz = 16;    // entries per row / column (two Givens stages)

template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
    return __builtin_nontemporal_load(p);
}

// Products val[k] * vec[idx[k]] of the entries [beg, end) of one wave's tile
// (at most kTile * kMaxNnz) into the wave's LDS slice.  All index and value
// loads are issued before the gathers, and all gathers before the stores,
// so a wave keeps up to 3 x 16 independent loads in flight.
template <typename T>
__device__ __forceinline__ void tile_products(const int32_t* __restrict__ idx, const T* __restrict__ val,
                                              const T* __restrict__ vec, int32_t beg, int32_t end,
                                              T* __restrict__ lds, int lane) {
    int32_t c[kMaxNnz];
    T v[kMaxNnz];
    T g[kMaxNnz];
#pragma unroll
    for (int q = 0; q < kMaxNnz; ++q) {
        const int32_t k = beg + q * kTile + lane;
        c[q] = (k < end) ? ld_stream(idx + k) : -1;
    }
#pragma unroll
    for (int q = 0; q < kMaxNnz; ++q) {
        const int32_t k = beg + q * kTile + lane;
        v[q] = (k < end) ? ld_stream(val + k) : T(0);
    }
#pragma unroll
    for (int q = 0; q < kMaxNnz; ++q) g[q] = (c[q] >= 0) ? vec[c[q]] : T(0);
#pragma unroll
    for (int q = 0; q < kMaxNnz; ++q)
        if (c[q] >= 0) lds[q * kTile + lane] = v[q] * g[q];
}

// Residual pass over one tile of 64 rows per wave.
// part[3*block + {0,1,2}] = sum r_x^2, sum r_y^2, sum b r_y (FP64).
// init = 1: r_y = r_x (first pass, beta_0 = 0, r_x,prev undefined).
template <typename T>
__global__ __launch_bounds__(L1LS_BLOCK) void k_residual(
    const int32_t* __restrict__ ptr, const int32_t* __restrict__ col, const T* __restrict__ val,
    const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ rx, T* __restrict__ ry, T beta,
    int64_t m, int init, double* __restrict__ part, const GapState* __restrict__ gs) {
    if (gs && gs->done) return;
    __shared__ T lds[L1LS_BLOCK / L1LS_WAVE][kTile * kMaxNnz];
    const int lane = threadIdx.x % L1LS_WAVE;
    const int wid = threadIdx.x / L1LS_WAVE;
    double v[3] = {0.0, 0.0, 0.0};
    const int64_t ntiles = (m + kTile - 1) / kTile;
    const int64_t wstride = (int64_t)gridDim.x * (L1LS_BLOCK / L1LS_WAVE);
    // uniform trip count across the block: every wave reaches the barriers
    const int64_t first = (int64_t)blockIdx.x * (L1LS_BLOCK / L1LS_WAVE);
    for (int64_t tb = first; tb < ntiles; tb += wstride) {
        const int64_t tile = tb + wid;
        const int64_t row0 = tile * kTile;
        const int64_t i = row0 + lane;
        const bool live = i < m;
        int32_t pb = 0, pe = 0;
        if (live) {
            pb = ptr[i];
            pe = ptr[i + 1];
        }
        const int64_t last = (row0 + kTile <= m) ? kTile - 1 : (m > row0 ? m - row0 - 1 : 0);
        const int32_t beg = __shfl(pb, 0, L1LS_WAVE);
        const int32_t end = __shfl(pe, (int)last, L1LS_WAVE);
        if (row0 < m) tile_products<T>(col, val, x, beg, end, lds[wid], lane);
        __syncthreads();
        if (live) {
            T acc = T(0);
            for (int32_t k = pb; k < pe; ++k) acc += lds[wid][k - beg];
            const T bi = b[i];
            const T r = acc - bi;
            const T yv = init ? r : (T(1) + beta) * r - beta * rx[i];
            rx[i] = r;
            ry[i] = yv;
            v[0] += (double)r * (double)r;
            v[1] += (double)yv * (double)yv;
            v[2] += (double)bi * (double)yv;
        }
        __syncthreads();
    }
    block_reduce_stats<3, 3>(v);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = v[0];
        part[3 * blockIdx.x + 1] = v[1];
        part[3 * blockIdx.x + 2] = v[2];
    }
}

// Transpose pass with the prox step over one tile of 64 columns per wave.
// xc = x_{k-1}; xp = x_{k-2} on entry and x_k on exit (same slot).
// part[2*block + {0,1}] = max |g|, sum |x_k|.
template <typename T>
__global__ __launch_bounds__(L1LS_BLOCK) void k_transpose_prox(
    const int32_t* __restrict__ ptr, const int32_t* __restrict__ row, const T* __restrict__ val,
    const T* __restrict__ ry, const T* __restrict__ xc, T* __restrict__ xp, T beta, T L, T thr,
    int64_t n, double* __restrict__ part, const GapState* __restrict__ gs) {
    if (gs && gs->done) return;
    __shared__ T lds[L1LS_BLOCK / L1LS_WAVE][kTile * kMaxNnz];
    const int lane = threadIdx.x % L1LS_WAVE;
    const int wid = threadIdx.x / L1LS_WAVE;
    double v[2] = {0.0, 0.0};  // sum |x_k|, max |g|
    const int64_t ntiles = (n + kTile - 1) / kTile;
    const int64_t wstride = (int64_t)gridDim.x * (L1LS_BLOCK / L1LS_WAVE);
    const int64_t first = (int64_t)blockIdx.x * (L1LS_BLOCK / L1LS_WAVE);
    for (int64_t tb = first; tb < ntiles; tb += wstride) {
        const int64_t tile = tb + wid;
        const int64_t col0 = tile * kTile;
        const int64_t j = col0 + lane;
        const bool live = j < n;
        int32_t pb = 0, pe = 0;
        if (live) {
            pb = ptr[j];
            pe = ptr[j + 1];
        }
        const int64_t last = (col0 + kTile <= n) ? kTile - 1 : (n > col0 ? n - col0 - 1 : 0);
        const int32_t beg = __shfl(pb, 0, L1LS_WAVE);
        const int32_t end = __shfl(pe, (int)last, L1LS_WAVE);
        if (col0 < n) tile_products<T>(row, val, ry, beg, end, lds[wid], lane);
        __syncthreads();
        if (live) {
            T acc = T(0);
            for (int32_t k = pb; k < pe; ++k) acc += lds[wid][k - beg];
            const T xcur = xc[j];
            const T y = xcur + beta * (xcur - xp[j]);
            const T xn = soft_threshold<T>(y - acc / L, thr);
            xp[j] = xn;
            v[0] += fabs((double)xn);
            v[1] = fmax(v[1], fabs((double)acc));
        }
        __syncthreads();
    }
    block_reduce_stats<2, 1>(v);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x + 0] = v[1];
        part[2 * blockIdx.x + 1] = v[0];
    }
}

// Duality gap at x_k (primal) and u = theta r_y,k (dual), from the partials:
//   P = tau ||x_k||_1 + 0.5 ||r_x,k||^2,
//   theta = min(1, tau / ||A^T r_y,k||_inf),
//   D = -0.5 theta^2 ||r_y,k||^2 - theta b^T r_y,k,
//   gap = (P - D) / |P|.
// One workgroup; fixed-order sums.
__global__ __launch_bounds__(1024) void k_gap(
    const double* __restrict__ k1_cur, const double* __restrict__ k1_prev, int g1,
    const double* __restrict__ k2, int g2, double tau, double tol, int64_t iter, GapState* gs) {
    if (gs->done) return;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // rr, ryy, bry, l1 | ginf
    for (int b = threadIdx.x; b < g1; b += blockDim.x) {
        v[0] += k1_cur[3 * b + 0];
        v[1] += k1_prev[3 * b + 1];
        v[2] += k1_prev[3 * b + 2];
    }
    for (int b = threadIdx.x; b < g2; b += blockDim.x) {
        v[3] += k2[2 * b + 1];
        v[4] = fmax(v[4], k2[2 * b + 0]);
    }
    block_reduce_stats<5, 4>(v);
    if (threadIdx.x == 0) {
        const double P = tau * v[3] + 0.5 * v[0];
        const double theta = (v[4] <= tau) ? 1.0 : tau / v[4];
        const double D = -0.5 * theta * theta * v[1] - theta * v[2];
        const double gap = (P - D) / fabs(P);
        gs->P = P;
        gs->D = D;
        gs->gap = gap;
        gs->ginf = v[4];
        gs->l1 = v[3];
        gs->rr = v[0];
        gs->iter = iter;
        const bool finite = (P == P) && (D == D) && (P - P == 0.0) && (D - D == 0.0);
        if (!finite) {
            gs->nonfinite = 1;
            gs->done = 1;
        } else if (gap <= tol) {
            gs->conv_iter = iter;
            gs->done = 1;
        }
    }
}

// Plain segmented SpMV: out[i] = sum_k val[k] in[idx[k]] over row/col i.
template <typename T, int W>
__global__ __launch_bounds__(L1LS_BLOCK) void k_spmv(const int32_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ idx,
                                                     const T* __restrict__ val, const T* __restrict__ in,
                                                     T* __restrict__ out, int64_t rows) {
    const int lane = threadIdx.x % W;
    const int64_t nseg = (int64_t)gridDim.x * (blockDim.x / W);
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / W; i < rows; i += nseg) {
        const int32_t beg = ptr[i], end = ptr[i + 1];
        T acc = T(0);
        for (int32_t k = beg + lane; k < end; k += W) acc += val[k] * in[idx[k]];
        acc = segment_sum<W>(acc);
        if (lane == 0) out[i] = acc;
    }
}

}  // namespace l1ls
