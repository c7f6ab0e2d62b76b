// Streaming kernels of the FISTA hot path (section 8.1, FISTA on problem
// (1)) over the stored operator:
//   residual pass  (CSR):  r_x = A x_k - b,  r_y = (1+beta_k) r_x - beta_k r_x,prev
//   transpose pass (CSC):  g = A^T r_y,  y = x_{k-1} + beta (x_{k-1} - x_{k-2}),
//                          x_k = soft(y - g/L, tau/L)
// plus FP64 partial statistics for the duality gap.  Each wave owns a tile
// of 64 consecutive rows (columns), one per lane: the tile's index and value
// loads and gathers are issued together, the products staged in LDS, and
// each lane sums its own row in storage order.  One workgroup (four waves)
// writes one slot of the partial arrays, and every reduction runs in a fixed
// order (bitwise reproducible).  k_spmv, the plain product, uses segments of
// W lanes per row with a grid-stride loop.
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

template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v) {
    __builtin_nontemporal_store(v, p);
}

// Element `i` of a device array addressed as base + 32-bit byte offset, so
// that the load takes its base from scalar registers (one VGPR per address).
// Valid for arrays below 4 GiB.
template <typename T>
__device__ __forceinline__ T ld_off32(const T* __restrict__ base, int32_t i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)i * (uint32_t)sizeof(T));
}

// Products val[k] * vec[idx[k]] of the entries [beg, beg + cnt) of one wave's
// tile (cnt <= kTile * kMaxNnz) into the wave's LDS slice.  The first
// NQ * 64 entries are handled without branches: lanes past the end load the
// last entry again (in bounds) and store a zero product, so the NQ index
// loads, NQ value loads and NQ gathers of a lane are all in flight together.
// The tile's base pointers are wave-uniform (scalar registers); per-lane
// offsets are 32-bit.  Entries beyond NQ * 64 go through a tail loop.
template <typename T>
__device__ __forceinline__ T ld_maybe_nt(const T* p, bool nt) {
    return nt ? __builtin_nontemporal_load(p) : *p;
}

template <typename T, int NQ, bool NT = true>
__device__ __forceinline__ void tile_products(const int32_t* __restrict__ idx, const T* __restrict__ val,
                                              const T* __restrict__ vec, int32_t beg, int32_t cnt,
                                              T* __restrict__ lds, int lane) {
    if (cnt <= 0) return;  // wave-uniform
    const int32_t* __restrict__ ib = idx + beg;
    const T* __restrict__ vb = val + beg;
    const int32_t last = cnt - 1;
    int32_t c[NQ];
    T v[NQ];
    T g[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) c[q] = ld_maybe_nt(ib + min(q * kTile + lane, last), NT);
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = ld_maybe_nt(vb + min(q * kTile + lane, last), NT);
#pragma unroll
    for (int q = 0; q < NQ; ++q) g[q] = ld_off32(vec, c[q]);
#pragma unroll
    for (int q = 0; q < NQ; ++q) lds[q * kTile + lane] = (q * kTile + lane <= last) ? v[q] * g[q] : T(0);
    for (int32_t k = NQ * kTile + lane; k <= last; k += kTile) lds[k] = vb[k] * ld_off32(vec, ib[k]);
}

// Workgroup index under XCD placement: workgroups are dispatched to the 8
// XCDs in turn (b, b + 8, ... on one XCD); with XCD set, XCD x takes one
// contiguous range of the logical indices instead, so the workgroups of one
// window of a windowed gather (window.hip) share one L2.
template <bool XCD>
__device__ __forceinline__ int64_t placed_block() {
    const int64_t b = blockIdx.x;
    if (!XCD) return b;
    const int64_t G = gridDim.x, q = G / 8, r = G % 8, x = b % 8;
    return x * q + (x < r ? x : r) + b / 8;
}

// Residual pass: one tile of 64 rows per wave, one wave-tile per launch slot.
// part[3*block + {0,1,2}] = sum r_x^2, sum r_y^2, sum b r_y (FP64).
// init = 1: r_y = r_x (first pass, beta_0 = 0, r_x,prev undefined).
// NQ, NT: the tile schedule (entries per lane issued together; nontemporal
// index and value loads), chosen by the autotuner; every choice computes the
// same values in the same order.
template <typename T, int NQ = 10, bool NT = true, bool XCD = false>
__global__ __launch_bounds__(L1LS_BLOCK) void k_residual(
    const int32_t* __restrict__ ptr, const int32_t* __restrict__ col, const T* __restrict__ val,
    const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ rx, T* __restrict__ ry, T beta,
    int64_t m, int init, double* __restrict__ part, const GapState* __restrict__ gs, int stats) {
    // Once the gap test has passed, the pass changes nothing.  The flag is
    // read together with the first loads and only guards the stores, so it
    // adds no round trip to a wave's critical path.
    const int32_t done = gs ? __builtin_nontemporal_load(&gs->done) : 0;
    __shared__ T lds[L1LS_BLOCK / L1LS_WAVE][kTile * kMaxNnz];
    const int lane = threadIdx.x % L1LS_WAVE;
    const int wid = threadIdx.x / L1LS_WAVE;
    const int64_t blk = placed_block<XCD>();
    const int64_t row0 = (blk * (L1LS_BLOCK / L1LS_WAVE) + wid) * kTile;
    const int64_t i = row0 + lane;
    const bool live = i < m;
    int32_t pb = 0, pe = 0;
    T bi = T(0), rprev = T(0);
    if (live) {
        pb = ptr[i];
        pe = ptr[i + 1];
        // epilogue operands do not depend on the products: load them now
        bi = __builtin_nontemporal_load(b + i);
        if (!init) rprev = __builtin_nontemporal_load(rx + i);
    }
    const int lastlane = (row0 + kTile <= m) ? kTile - 1 : (m > row0 ? (int)(m - row0 - 1) : 0);
    const int32_t beg = __builtin_amdgcn_readfirstlane(__shfl(pb, 0, L1LS_WAVE));
    const int32_t end = __builtin_amdgcn_readfirstlane(__shfl(pe, lastlane, L1LS_WAVE));
    if (row0 < m) tile_products<T, NQ, NT>(col, val, x, beg, end - beg, lds[wid], lane);
    __syncthreads();
    double v[3] = {0.0, 0.0, 0.0};
    if (live && !done) {
        T acc = T(0);
        for (int32_t k = pb - beg; k < pe - beg; ++k) acc += lds[wid][k];
        const T r = acc - bi;
        const T yv = init ? r : (T(1) + beta) * r - beta * rprev;
        st_stream(rx + i, r);
        st_stream(ry + i, yv);
        v[0] = (double)r * (double)r;
        v[1] = (double)yv * (double)yv;
        v[2] = (double)bi * (double)yv;
    }
    if (!stats) return;  // launch-uniform: the gap test does not read this pass
    block_reduce_stats<3, 3>(v);
    if (threadIdx.x == 0 && !done) {
        part[3 * blk + 0] = v[0];
        part[3 * blk + 1] = v[1];
        part[3 * blk + 2] = v[2];
    }
}

// Transpose pass with the prox step: one tile of 64 columns per wave.
// xc = x_{k-1}; xp = x_{k-2} on entry and x_k on exit (same slot).
// part[2*block + {0,1}] = max |g|, sum |x_k|.  NQ, NT as for k_residual.
template <typename T, int NQ = 16, bool NT = true, bool XCD = false>
__global__ __launch_bounds__(L1LS_BLOCK) void k_transpose_prox(
    const int32_t* __restrict__ ptr, const int32_t* __restrict__ row, const T* __restrict__ val,
    const T* __restrict__ ry, const T* __restrict__ xc, T* __restrict__ xp, T beta, T L, T thr,
    int64_t n, double* __restrict__ part, const GapState* __restrict__ gs, int stats) {
    const int32_t done = gs ? __builtin_nontemporal_load(&gs->done) : 0;  // guards the stores only
    __shared__ T lds[L1LS_BLOCK / L1LS_WAVE][kTile * kMaxNnz];
    const int lane = threadIdx.x % L1LS_WAVE;
    const int wid = threadIdx.x / L1LS_WAVE;
    const int64_t blk = placed_block<XCD>();
    const int64_t col0 = (blk * (L1LS_BLOCK / L1LS_WAVE) + wid) * kTile;
    const int64_t j = col0 + lane;
    const bool live = j < n;
    int32_t pb = 0, pe = 0;
    T xcur = T(0), xprev = T(0);
    if (live) {
        pb = ptr[j];
        pe = ptr[j + 1];
        xcur = __builtin_nontemporal_load(xc + j);
        xprev = __builtin_nontemporal_load(xp + j);
    }
    const int lastlane = (col0 + kTile <= n) ? kTile - 1 : (n > col0 ? (int)(n - col0 - 1) : 0);
    const int32_t beg = __builtin_amdgcn_readfirstlane(__shfl(pb, 0, L1LS_WAVE));
    const int32_t end = __builtin_amdgcn_readfirstlane(__shfl(pe, lastlane, L1LS_WAVE));
    if (col0 < n) tile_products<T, NQ, NT>(row, val, ry, beg, end - beg, lds[wid], lane);
    __syncthreads();
    double v[2] = {0.0, 0.0};  // sum |x_k|, max |g|
    if (live && !done) {
        T acc = T(0);
        for (int32_t k = pb - beg; k < pe - beg; ++k) acc += lds[wid][k];
        const T y = xcur + beta * (xcur - xprev);
        const T xn = soft_threshold<T>(y - acc / L, thr);
        st_stream(xp + j, xn);
        v[0] = fabs((double)xn);
        v[1] = fabs((double)acc);
    }
    if (!stats) return;  // launch-uniform
    block_reduce_stats<2, 1>(v);
    if (threadIdx.x == 0 && !done) {
        part[2 * blk + 0] = v[1];
        part[2 * blk + 1] = v[0];
    }
}

// Duality gap at x_k (primal) and u = theta r_y,k (dual), from the partials:
//   P = tau ||x_k||_1 + 0.5 ||r_x,k||^2,
//   theta = min(1, tau / ||A^T r_y,k||_inf),
//   D = -0.5 theta^2 ||r_y,k||^2 - theta b^T r_y,k,
//   gap = (P - D) / |P|.
// One workgroup; fixed-order sums.
// The five gap sums (rr, ryy, bry, l1 | ginf) over the workgroup partials
// [b1, e1) of the residual passes and [b2, e2) of the transpose pass, in a
// fixed order (strided per thread, then block_reduce_stats).
__device__ __forceinline__ void gap_sums(const double* __restrict__ k1_cur, const double* __restrict__ k1_prev,
                                         int b1, int e1, const double* __restrict__ k2, int b2, int e2,
                                         double (&v)[5]) {
    for (int b = b1 + (int)threadIdx.x; b < e1; b += blockDim.x) {
        v[0] += k1_cur[3 * b + 0];
        v[1] += k1_prev[3 * b + 1];
        v[2] += k1_prev[3 * b + 2];
    }
    for (int b = b2 + (int)threadIdx.x; b < e2; b += blockDim.x) {
        v[3] += k2[2 * b + 1];
        v[4] = fmax(v[4], k2[2 * b + 0]);
    }
    block_reduce_stats<5, 4>(v);
}

__device__ __forceinline__ void gap_finish(const double (&v)[5], double tau, double tol, int64_t iter, GapState* gs);

static __global__ __launch_bounds__(1024) void k_gap(
    const double* __restrict__ k1_cur, const double* __restrict__ k1_prev, int g1,
    const double* __restrict__ k2, int g2, double tau, double tol, int64_t iter, GapState* gs) {
    if (gs->done) return;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // rr, ryy, bry, l1 | ginf
    gap_sums(k1_cur, k1_prev, 0, g1, k2, 0, g2, v);
    if (threadIdx.x == 0) gap_finish(v, tau, tol, iter, gs);
}

// Large grids (hundreds of thousands of partials): a first stage of
// kGapStages workgroups, each over a contiguous share of the partials, then
// k_gap_final over their kGapStages x 5 sums.
constexpr int kGapStages = 256;

static __global__ __launch_bounds__(1024) void k_gap_stage(
    const double* __restrict__ k1_cur, const double* __restrict__ k1_prev, int g1,
    const double* __restrict__ k2, int g2, double* __restrict__ out, const GapState* __restrict__ gs) {
    if (gs->done) return;
    const int c1 = (g1 + kGapStages - 1) / kGapStages, c2 = (g2 + kGapStages - 1) / kGapStages;
    const int b = blockIdx.x;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    gap_sums(k1_cur, k1_prev, min(b * c1, g1), min((b + 1) * c1, g1), k2, min(b * c2, g2), min((b + 1) * c2, g2), v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < 5; ++i) out[5 * b + i] = v[i];
    }
}

static __global__ __launch_bounds__(1024) void k_gap_final(const double* __restrict__ st, double tau, double tol,
                                                           int64_t iter, GapState* gs) {
    if (gs->done) return;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < kGapStages; b += blockDim.x) {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] += st[5 * b + i];
        v[4] = fmax(v[4], st[5 * b + 4]);
    }
    block_reduce_stats<5, 4>(v);
    if (threadIdx.x == 0) gap_finish(v, tau, tol, iter, gs);
}

__device__ __forceinline__ void gap_finish(const double (&v)[5], double tau, double tol, int64_t iter, GapState* gs) {
    {
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
        } else if (tol > 0.0 && gap <= tol) {
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
