// Matrix-free FISTA passes (section 4, Algorithms MvPA and MvPAt: A as the
// operator Q Sigma G^T from the rotation triplets, without a stored A) in
// stage order.
//
// In stage order (position p of a side holds original index pi(p)) stage 1
// pairs positions (2k, 2k+1) and stage 2 pairs (2k+1, 2k+2 mod N), so every
// Givens stage is a local stencil.  The only non-local step is Sigma, which
// links n-position a and m-position i when pi_n(a) = pi_m(i):
//   emb[i] = a (or -1 when pi_m(i) >= n),  sig[i] = sigma_{pi_m(i)} (0 when
//   inactive); inv[a] = rank, among the active m-positions, of the i linked
//   to a.
// A x   = Q (Sigma (G^T x)):  pass 1 (n side) w_a = sigma_a (G^T x)_a, written
//                             in n order; pass 2 (m side) gathers
//                             z_i = w_{emb_i}, r = Q z, fused with the
//                             residual/momentum epilogue.
// A^T r = G (Sigma^T (Q^T r)): pass 1 (m side) v = sig_i (Q^T r)_i at the
//                             active m-positions, written compactly at their
//                             rank (n long); pass 2 (n side) gathers
//                             t_a = v_{inv_a}, g = G t, fused with the
//                             gradient step, prox, momentum.
// The embedding is a random permutation, so its accesses are random: they
// are made as gathers (one per position, staged in LDS for the stencil that
// follows), never as scattered stores.  Every XCD caches the whole vector it
// gathers from, so the compact v (n values instead of m) halves that cost on
// the A^T side.  The stores into the compact v keep position order, so they
// stay near-coalesced.  Each thread owns one rotation pair of the last stage
// it applies and reads the 4 consecutive positions that feed it.  The rank
// of an active m-position is the workgroup's base (cbase: active positions
// before the workgroup's first) plus a ballot count within the workgroup, so
// no per-position table is read for it.
#include "common.hpp"
#include "kernels.hpp"

using namespace l1ls;

namespace {

template <typename T>
struct MfTabs {
    const T* csn[L1LS_MAX_ROUNDS];  // n side, per stage: (c, s) per pair
    const T* csm[L1LS_MAX_ROUNDS];  // m side
    const int32_t* emb;             // m
    const int32_t* inv;             // n: rank of the linked m-position among the active ones
    const int32_t* cbase;           // per workgroup of the m side: active positions before it
    const int32_t* gm;              // m side's gather index into its source: emb, or the window slots
    const int32_t* gn;              // n side's gather index: inv, or the window slots
    int xcd;                        // windowed gathers: place each XCD's workgroups on one range (mf_block)
    const T* sig;                   // m: sigma at m-positions (0 if inactive)
    const T* sig_n;                 // n: sigma at n-positions
    int64_t n, m;
};

template <typename T>
struct CS {
    T c, s;
};

template <typename T>
__device__ __forceinline__ CS<T> cs_of(const T* tab, int64_t k) {
    return CS<T>{tab[2 * k], tab[2 * k + 1]};
}

__device__ __forceinline__ int64_t wrap(int64_t p, int64_t N) { return p < 0 ? p + N : (p >= N ? p - N : p); }

// G(f,g): (zf, zg) -> (c zf - s zg, s zf + c zg); transpose: (c zf + s zg, -s zf + c zg)
template <typename T, typename TT>
__device__ __forceinline__ void rot(CS<TT> rt, T zf, T zg, bool transpose, T& of, T& og) {
    const CS<T> r{(T)rt.c, (T)rt.s};  // tables of type TT, vectors of type T
    if (transpose) {
        of = r.c * zf + r.s * zg;
        og = -r.s * zf + r.c * zg;
    } else {
        of = r.c * zf - r.s * zg;
        og = r.s * zf + r.c * zg;
    }
}

// Position p + q of a side of N positions, reduced mod N (q >= 0 small).
__device__ __forceinline__ int64_t ring(int64_t p, int64_t N) {
    if (p >= N) p -= N;
    if (p >= N) p %= N;  // only for sides shorter than a block's reach
    return p;
}

// A workgroup's gather into LDS: dst[q] = src[idx[p]] for the 2B + 2H
// positions p = 2 k0 - H + q (mod N), 0 where idx[p] < 0 (an inactive
// position).  All of a thread's index loads are issued before its gathers,
// and all gathers before the LDS stores, so the dependent pairs of loads of
// its two or three positions are in flight together.
template <typename T, int B, int H>
__device__ __forceinline__ void gather_block(const T* __restrict__ src, const int32_t* __restrict__ idx, int64_t k0,
                                             int64_t N, T* dst) {
    constexpr int Q = 2 * B + 2 * H;
    constexpr int NQ = (Q + B - 1) / B;
    int32_t a[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int q = threadIdx.x + u * B;
        a[u] = (q < Q) ? idx[ring(2 * k0 - H + q + N, N)] : -1;
    }
    T z[NQ];
#pragma unroll
    for (int u = 0; u < NQ; ++u) z[u] = (a[u] >= 0) ? ld_off32(src, a[u]) : T(0);
#pragma unroll
    for (int u = 0; u < NQ; ++u) {
        const int q = threadIdx.x + u * B;
        if (q < Q) dst[q] = z[u];
    }
}

// Workgroup index of a matrix-free pass.  Workgroups are handed to the 8
// XCDs in turn (b, b+8, ... on one XCD); with xcd set, XCD x takes one
// contiguous range of the pairs instead, so the workgroups of one gather
// window share one L2, which then fetches that window's segment once.
__device__ __forceinline__ int64_t mf_block(int xcd) {
    const int64_t b = blockIdx.x;
    if (!xcd) return b;
    const int64_t G = gridDim.x, q = G / 8, r = G % 8, x = b % 8;
    return x * q + (x < r ? x : r) + b / 8;
}

// Rank of the m-positions 2k and 2k+1 (k = blk B + threadIdx.x, the
// thread's stage-1 pair) among the active ones, or -1 where inactive.  Every
// thread of the workgroup takes part, between two phases the caller puts a
// __syncthreads: rank_count publishes each wave's count of active positions
// in ws, rank_of adds the lower waves' counts to the workgroup's base.
struct PairRank {
    int32_t pre;  // active positions of lower lanes of the wave
    bool a0, a1;
};
constexpr int kMfWaves = L1LS_BLOCK / 64;
__device__ __forceinline__ PairRank rank_count(const int32_t* __restrict__ emb, int64_t kc, bool mine,
                                               int32_t* ws) {
    const int2 e = *reinterpret_cast<const int2*>(emb + 2 * kc);  // 2kc even: 8-byte aligned
    PairRank r;
    r.a0 = mine && e.x >= 0;
    r.a1 = mine && e.y >= 0;
    const uint64_t b0 = __ballot(r.a0), b1 = __ballot(r.a1);
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    r.pre = __popcll(b0 & below) + __popcll(b1 & below);
    if (lane == 0) ws[threadIdx.x >> 6] = __popcll(b0) + __popcll(b1);
    return r;
}
__device__ __forceinline__ void rank_of(const PairRank& r, const int32_t* __restrict__ cbase, int64_t blk,
                                        const int32_t* ws, int32_t& ci0, int32_t& ci1) {
    int32_t base = cbase[blk] + r.pre;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int w = 0; w < kMfWaves; ++w)
        if (w < wave) base += ws[w];
    ci0 = r.a0 ? base : -1;
    ci1 = r.a1 ? base + (r.a0 ? 1 : 0) : -1;
}

// w = Sigma_n G^T x in n-stage order (sigma at n-positions, 0 where the
// column has no sigma).  R = 2: G^T = S_1^T S_2^T (S_2^T first); thread k
// handles stage-1 pair (2k, 2k+1) from x at 2k-1 .. 2k+2.
template <typename T, int R, typename TT = T>
__global__ __launch_bounds__(L1LS_BLOCK) void k_mf_gt(const T* __restrict__ x, T* __restrict__ w, MfTabs<TT> tb,
                                                       const int32_t* __restrict__ done) {
    if (done && *done) return;  // the solver's converged flag (launch-uniform)
    const int64_t n = tb.n, np = n / 2;
    const int64_t k = (int64_t)blockIdx.x * L1LS_BLOCK + threadIdx.x;
    if (k >= np) return;
    T z0 = x[2 * k], z1 = x[2 * k + 1];
    if (R == 2) {
        const T xm = x[wrap(2 * k - 1, n)], xp = x[wrap(2 * k + 2, n)];
        T a, b;
        rot(cs_of(tb.csn[1], wrap(k - 1, np)), xm, z0, true, a, b);  // 2k is second of stage-2 pair k-1
        const T z0n = b;
        rot(cs_of(tb.csn[1], k), z1, xp, true, a, b);                // 2k+1 is first of stage-2 pair k
        z0 = z0n;
        z1 = a;
    }
    T o0, o1;
    rot(cs_of(tb.csn[0], k), z0, z1, true, o0, o1);
    w[2 * k] = (T)tb.sig_n[2 * k] * o0;
    w[2 * k + 1] = (T)tb.sig_n[2 * k + 1] * o1;
}

// Residual pass fused with the m side of the next transpose product.
// r_x = Q z - b and r_y = (1+beta) r_x - beta r_x,prev with z_i = w[emb[i]]
// (0 at inactive m-positions), then v = Sigma_m Q^T r_y written in m order.
// A workgroup owns pairs k0 .. k0+B-1.  R = 2: Q = S~_2 S~_1; stage-2 pair j
// yields r at (2j+1, 2j+2) from z at 2j .. 2j+3, and the Q^T of stage-1 pair
// k reads r_y at 2k-1 .. 2k+2, so the workgroup also evaluates stage-2 pair
// k0-1 (its left neighbour's, not stored) and gathers z at 2k0-2 ..
// 2k0+2B+1.  r_y never leaves LDS.  R = 1: pair k only.  r_x,prev (rxp) and
// r_x (rx) are separate buffers: a neighbour's r_x,prev is read for the halo
// while its owner writes r_x.
// MODE selects what the pass is for:
//   kMfFista   the FISTA residual pass above;
//   kMfProduct rx = A x only (b = 0, no v);
//   kMfNormal  vm = Sigma_m Q^T (A x) only (b = 0, rx not written): the
//              m side of A^T A x for the second-order path.
constexpr int kMfFista = 0, kMfProduct = 1, kMfNormal = 2;
template <typename T, int R, int MODE = kMfFista, typename TT = T>
__global__ __launch_bounds__(L1LS_BLOCK) void k_mf_res_qt(const T* __restrict__ w, const T* __restrict__ b,
                                                           const T* __restrict__ rxp, T* __restrict__ rx,
                                                           T* __restrict__ vm, T beta,
                                                           int init, MfTabs<TT> tb, double* __restrict__ part,
                                                           const int32_t* __restrict__ done, int stats) {
    constexpr int B = L1LS_BLOCK;
    constexpr int H = (R == 2) ? 2 : 0;  // halo positions on the left
    __shared__ T zl[2 * B + 2 * H];
    __shared__ T yl[2 * B + H];  // r_y at positions 2k0 - H/2 .. (R = 2: from 2k0-1)
    if (done && *done) return;  // the solver's converged flag (launch-uniform)
    const int64_t m = tb.m, mp = m / 2;
    const int64_t blk = mf_block(tb.xcd);
    const int64_t k0 = blk * B;
    const int t = threadIdx.x;
    const int64_t k = k0 + t;
    const bool mine = k < mp;
    const int64_t kc = mine ? k : mp - 1;  // threads past the end load in bounds, use nothing
    // Everything that does not depend on the gather is loaded first, so that
    // its latency overlaps the gather's: the rotations of the thread's pairs,
    // b and r_x,prev at its two outputs, sigma at its stage-1 pair.
    const CS<TT> c1 = cs_of(tb.csm[0], kc);  // stage-1 pair k
    CS<TT> c1n{TT(0), TT(0)}, c2{TT(0), TT(0)}, c2m{TT(0), TT(0)};
    int64_t ps[2];
    if (R == 2) {
        c1n = cs_of(tb.csm[0], wrap(kc + 1, mp));  // stage-1 pair k+1
        c2 = cs_of(tb.csm[1], kc);                 // stage-2 pair k
        if (MODE != kMfProduct) c2m = cs_of(tb.csm[1], wrap(kc - 1, mp));  // stage-2 pair k-1, for Q^T
        ps[0] = 2 * kc + 1;
        ps[1] = wrap(2 * kc + 2, m);
    } else {
        ps[0] = 2 * kc;
        ps[1] = 2 * kc + 1;
    }
    T bo[2] = {T(0), T(0)}, rpo[2] = {T(0), T(0)};
    if (MODE == kMfFista) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            bo[e] = b[ps[e]];
            if (!init) rpo[e] = rxp[ps[e]];
        }
    }
    T s0 = T(0), s1 = T(0);
    __shared__ int32_t ws[kMfWaves];
    PairRank pr{0, false, false};
    if (MODE != kMfProduct) {
        s0 = (T)tb.sig[2 * kc];
        s1 = (T)tb.sig[2 * kc + 1];
        pr = rank_count(tb.gm, kc, mine, ws);
    }
    gather_block<T, B, H>(w, tb.gm, k0, m, zl);
    __syncthreads();
    double v[3] = {0.0, 0.0, 0.0};
    if (R == 2) {
        // thread 0 also evaluates the left neighbour's stage-2 pair k0-1 (not
        // stored): Q^T of stage-1 pair k0 reads r_y at 2k0-1
        if (t == 0 && MODE != kMfProduct) {
            const int64_t j = wrap(k0 - 1, mp);
            T a, u1, u2, bb, rf, rg;
            rot(cs_of(tb.csm[0], j), zl[0], zl[1], false, a, u1);
            rot(cs_of(tb.csm[0], wrap(j + 1, mp)), zl[2], zl[3], false, u2, bb);
            rot(cs_of(tb.csm[1], j), u1, u2, false, rf, rg);
            const int64_t pn[2] = {2 * j + 1, wrap(2 * j + 2, m)};
            const T rr[2] = {rf, rg};
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const T bi = (MODE == kMfFista) ? b[pn[e]] : T(0);
                const T r = rr[e] - bi;
                yl[e] = (init || MODE != kMfFista) ? r : (T(1) + beta) * r - beta * rxp[pn[e]];
            }
        }
        if (mine) {
            // own stage-2 pair k: r at 2k+1, 2k+2 from z at 2k .. 2k+3
            const int q0 = 2 * t + 2;
            T a, u1, u2, bb, rf, rg;
            rot(c1, zl[q0], zl[q0 + 1], false, a, u1);
            rot(c1n, zl[q0 + 2], zl[q0 + 3], false, u2, bb);
            rot(c2, u1, u2, false, rf, rg);
            const T rr[2] = {rf, rg};
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const T r = rr[e] - bo[e];
                const T yv = (init || MODE != kMfFista) ? r : (T(1) + beta) * r - beta * rpo[e];
                yl[q0 + e] = yv;
                if (MODE != kMfNormal) rx[ps[e]] = r;
                v[0] += (double)r * (double)r;
                v[1] += (double)yv * (double)yv;
                v[2] += (double)bo[e] * (double)yv;
            }
        }
    } else if (mine) {
        T rf, rg;
        rot(c1, zl[2 * t], zl[2 * t + 1], false, rf, rg);
        const T rr[2] = {rf, rg};
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const T r = rr[e] - bo[e];
            const T yv = (init || MODE != kMfFista) ? r : (T(1) + beta) * r - beta * rpo[e];
            yl[2 * t + e] = yv;
            if (MODE != kMfNormal) rx[ps[e]] = r;
            v[0] += (double)r * (double)r;
            v[1] += (double)yv * (double)yv;
            v[2] += (double)bo[e] * (double)yv;
        }
    }
    __syncthreads();
    if (MODE != kMfProduct && mine) {
        // v for stage-1 pair k; pairs with both positions inactive are not read
        if (s0 != T(0) || s1 != T(0)) {
            T z0, z1;
            if (R == 2) {
                T a, bq;
                rot(c2m, yl[2 * t], yl[2 * t + 1], true, a, bq);  // r_y at 2k-1, 2k
                const T z0n = bq;
                rot(c2, yl[2 * t + 2], yl[2 * t + 3], true, a, bq);  // r_y at 2k+1, 2k+2
                z0 = z0n;
                z1 = a;
            } else {
                z0 = yl[2 * t];
                z1 = yl[2 * t + 1];
            }
            T o0, o1;
            rot(c1, z0, z1, true, o0, o1);
            int32_t ci0, ci1;
            rank_of(pr, tb.cbase, blk, ws, ci0, ci1);
            if (ci0 >= 0) vm[ci0] = s0 * o0;
            if (ci1 >= 0) vm[ci1] = s1 * o1;
        }
    }
    if (!stats) return;
    block_reduce_stats<3, 3>(v);
    if (threadIdx.x == 0) {
        part[3 * blk + 0] = v[0];
        part[3 * blk + 1] = v[1];
        part[3 * blk + 2] = v[2];
    }
}

// Transpose pass fused with the n side of the next residual product.
// g = G t with t_a = v[inv[a]]; y = x_{k-1} + beta (x_{k-1} - x_{k-2}),
// x_k = soft(y - g/L, tau/L) written to xo (a buffer other than xp: a
// neighbour's x_{k-2} is read for the halo while its owner writes x_k); then
// w = Sigma_n G^T x_k written in n order.  The halo is as in k_mf_res_qt
// (R = 2: stage-2 pair k0-1 is evaluated again, not stored; t gathered at
// 2k0-2 .. 2k0+2B+1).  x_k of the workgroup's pairs stays in LDS for G^T.
template <typename T, int R>
__global__ __launch_bounds__(L1LS_BLOCK) void k_mf_prox_gt(const T* __restrict__ vm, const T* __restrict__ xc,
                                                            const T* __restrict__ xp, T* __restrict__ xo,
                                                            T* __restrict__ w, T beta, T L,
                                                            T thr, MfTabs<T> tb, double* __restrict__ part,
                                                            const GapState* __restrict__ gs, int stats) {
    constexpr int B = L1LS_BLOCK;
    constexpr int H = (R == 2) ? 2 : 0;
    __shared__ T tl[2 * B + 2 * H];
    __shared__ T xl[2 * B + H];
    const int32_t done = gs ? gs->done : 0;
    if (done) return;  // launch-uniform
    const int64_t n = tb.n, np = n / 2;
    const int64_t blk = mf_block(tb.xcd);
    const int64_t k0 = blk * B;
    // one position at a time: measured about 5% faster for this kernel than
    // gather_block's overlapped loads
    for (int q = threadIdx.x; q < 2 * B + 2 * H; q += B) {
        const int64_t p = ring(2 * k0 - H + q + n, n);
        tl[q] = ld_off32(vm, tb.gn[p]);
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int64_t k = k0 + t;
    double v[2] = {0.0, 0.0};  // sum |x_k|, max |g|
    if (R == 2) {
        for (int h = 0; h < (t == 0 ? 2 : 1); ++h) {
            const bool own = (h == 0);
            const int64_t j = own ? k : wrap(k0 - 1, np);
            if (own && j >= np) break;
            const int q0 = own ? 2 * t + 2 : 0;
            T a, u1, u2, bb, gf, gg;
            rot(cs_of(tb.csn[0], j), tl[q0], tl[q0 + 1], false, a, u1);
            rot(cs_of(tb.csn[0], wrap(j + 1, np)), tl[q0 + 2], tl[q0 + 3], false, u2, bb);
            rot(cs_of(tb.csn[1], j), u1, u2, false, gf, gg);
            const int64_t ps[2] = {2 * j + 1, wrap(2 * j + 2, n)};
            const T gv[2] = {gf, gg};
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int64_t jj = ps[e];
                const T xcur = xc[jj];
                const T y = xcur + beta * (xcur - xp[jj]);
                const T xn = soft_threshold<T>(y - gv[e] / L, thr);
                xl[(own ? 2 * t + 2 : 0) + e] = xn;
                if (own) {
                    xo[jj] = xn;
                    v[0] += fabs((double)xn);
                    v[1] = fmax(v[1], fabs((double)gv[e]));
                }
            }
        }
    } else if (k < np) {
        T gf, gg;
        rot(cs_of(tb.csn[0], k), tl[2 * t], tl[2 * t + 1], false, gf, gg);
        const int64_t ps[2] = {2 * k, 2 * k + 1};
        const T gv[2] = {gf, gg};
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int64_t jj = ps[e];
            const T xcur = xc[jj];
            const T y = xcur + beta * (xcur - xp[jj]);
            const T xn = soft_threshold<T>(y - gv[e] / L, thr);
            xl[2 * t + e] = xn;
            xo[jj] = xn;
            v[0] += fabs((double)xn);
            v[1] = fmax(v[1], fabs((double)gv[e]));
        }
    }
    __syncthreads();
    if (k < np) {
        T z0, z1;
        if (R == 2) {
            const T xm = xl[2 * t], xq = xl[2 * t + 3];  // x_k at 2k-1 and 2k+2
            T a, bq;
            rot(cs_of(tb.csn[1], wrap(k - 1, np)), xm, xl[2 * t + 1], true, a, bq);
            const T z0n = bq;
            rot(cs_of(tb.csn[1], k), xl[2 * t + 2], xq, true, a, bq);
            z0 = z0n;
            z1 = a;
        } else {
            z0 = xl[2 * t];
            z1 = xl[2 * t + 1];
        }
        T o0, o1;
        rot(cs_of(tb.csn[0], k), z0, z1, true, o0, o1);
        w[2 * k] = tb.sig_n[2 * k] * o0;
        w[2 * k + 1] = tb.sig_n[2 * k + 1] * o1;
    }
    if (!stats) return;
    block_reduce_stats<2, 1>(v);
    if (threadIdx.x == 0) {
        part[2 * blk + 0] = v[1];
        part[2 * blk + 1] = v[0];
    }
}

// v = Sigma_m Q^T y at the active m-positions, compact (the m side of A^T y
// on its own).  Thread k owns stage-1 pair k; R = 2: Q^T = S~_1^T S~_2^T
// reads y at 2k-1 .. 2k+2.  Threads past the end take part in the rank only.
template <typename T, int R>
__global__ __launch_bounds__(L1LS_BLOCK) void k_mf_qt(const T* __restrict__ y, T* __restrict__ vm, MfTabs<T> tb) {
    __shared__ int32_t ws[kMfWaves];
    const int64_t m = tb.m, mp = m / 2;
    const int64_t blk = mf_block(tb.xcd);
    const int64_t k0 = blk * L1LS_BLOCK + threadIdx.x;
    const bool mine = k0 < mp;
    const int64_t k = mine ? k0 : mp - 1;
    const PairRank pr = rank_count(tb.gm, k, mine, ws);
    __syncthreads();
    int32_t ci0, ci1;
    rank_of(pr, tb.cbase, blk, ws, ci0, ci1);
    if (!mine) return;
    T z0 = y[2 * k], z1 = y[2 * k + 1];
    if (R == 2) {
        const T ym = y[wrap(2 * k - 1, m)], yp = y[wrap(2 * k + 2, m)];
        T a, b;
        rot(cs_of(tb.csm[1], wrap(k - 1, mp)), ym, z0, true, a, b);  // 2k is second of stage-2 pair k-1
        const T z0n = b;
        rot(cs_of(tb.csm[1], k), z1, yp, true, a, b);                // 2k+1 is first of stage-2 pair k
        z0 = z0n;
        z1 = a;
    }
    T o0, o1;
    rot(cs_of(tb.csm[0], k), z0, z1, true, o0, o1);
    if (ci0 >= 0) vm[ci0] = tb.sig[2 * k] * o0;
    if (ci1 >= 0) vm[ci1] = tb.sig[2 * k + 1] * o1;
}

// The n side of A^T from the compact v: g = G t with t_a = v[inv[a]], with the
// Hessian epilogue of the PCG when p is given:
//   h = g + d p (d optional), h = 0 where mask is 0 (mask optional),
//   out = h, part[block] = sum p h (part optional);
// without p: out = g.  Gather and halo as in k_mf_prox_gt (R = 2: thread t
// owns stage-2 pair k0 + t, outputs at 2k+1 and 2k+2).
template <typename T, int R, typename TT = T>
__global__ __launch_bounds__(L1LS_BLOCK) void k_mf_g_hess(const T* __restrict__ vm, const T* __restrict__ p,
                                                           const T* __restrict__ d, const uint8_t* __restrict__ mask,
                                                           T* __restrict__ out, MfTabs<TT> tb,
                                                           double* __restrict__ part,
                                                           const int32_t* __restrict__ done) {
    constexpr int B = L1LS_BLOCK;
    constexpr int H = (R == 2) ? 2 : 0;
    __shared__ T tl[2 * B + 2 * H];
    if (done && *done) return;  // launch-uniform
    const int64_t n = tb.n, np = n / 2;
    const int64_t blk = mf_block(tb.xcd);
    const int64_t k0 = blk * B;
    const int t = threadIdx.x;
    const int64_t k = k0 + t;
    const bool mine = k < np;
    const int64_t kc = mine ? k : np - 1;  // threads past the end load in bounds, use nothing
    // operands independent of the gather first: rotations, p, d, mask
    const CS<TT> c1 = cs_of(tb.csn[0], kc);
    CS<TT> c1n{TT(0), TT(0)}, c2{TT(0), TT(0)};
    int64_t ps[2];
    if (R == 2) {
        c1n = cs_of(tb.csn[0], wrap(kc + 1, np));
        c2 = cs_of(tb.csn[1], kc);
        ps[0] = 2 * kc + 1;
        ps[1] = wrap(2 * kc + 2, n);
    } else {
        ps[0] = 2 * kc;
        ps[1] = 2 * kc + 1;
    }
    T pv[2] = {T(0), T(0)}, dv[2] = {T(0), T(0)};
    bool on[2] = {true, true};
    if (p) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            pv[e] = p[ps[e]];
            if (d) dv[e] = d[ps[e]];
            if (mask) on[e] = mask[ps[e]] != 0;
        }
    }
    gather_block<T, B, H>(vm, tb.gn, k0, n, tl);
    __syncthreads();
    double acc[1] = {0.0};
    if (mine) {
        T gv[2];
        if (R == 2) {
            const int q0 = 2 * t + 2;  // t at 2k .. 2k+3
            T a, u1, u2, bb;
            rot(c1, tl[q0], tl[q0 + 1], false, a, u1);
            rot(c1n, tl[q0 + 2], tl[q0 + 3], false, u2, bb);
            rot(c2, u1, u2, false, gv[0], gv[1]);
        } else {
            rot(c1, tl[2 * t], tl[2 * t + 1], false, gv[0], gv[1]);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            T h = gv[e];
            if (p) {
                if (d) h += dv[e] * pv[e];
                if (!on[e]) h = T(0);
                acc[0] += (double)pv[e] * (double)h;
            }
            out[ps[e]] = h;
        }
    }
    if (!part) return;  // launch-uniform
    block_reduce_stats<1, 1>(acc);
    if (threadIdx.x == 0) part[blk] = acc[0];
}

// ---- tables ------------------------------------------------------------------
__global__ void k_mf_emb(const int32_t* __restrict__ perm_m, const int32_t* __restrict__ pinv_n,
                         const double* __restrict__ sigma, int64_t n, int64_t m, int32_t* __restrict__ emb,
                         double* __restrict__ sig64, float* __restrict__ sig32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int32_t o = perm_m[i];
    const bool on = o < n;
    emb[i] = on ? pinv_n[o] : -1;
    const double sg = on ? sigma[o] : 0.0;
    sig64[i] = sg;
    sig32[i] = (float)sg;
}

__global__ void k_mf_active(const int32_t* __restrict__ perm_m, int64_t n, int64_t m, int32_t* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) flag[i] = perm_m[i] < n ? 1 : 0;
}

// cbase[g]: active m-positions before the first of workgroup g (positions
// 2 g B .. 2 g B + 2B - 1 of the m side); off = exclusive scan of the flags.
__global__ void k_mf_cbase(const int32_t* __restrict__ off, int64_t m, int64_t groups, int32_t* __restrict__ cbase) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < groups) cbase[g] = off[std::min<int64_t>(2 * g * L1LS_BLOCK, m)];
}

// inv[a]: rank, among the active m-positions, of the one linked to n-position a
__global__ void k_mf_inv(const int32_t* __restrict__ perm_n, const int32_t* __restrict__ pinv_m,
                         const int32_t* __restrict__ off, const double* __restrict__ sigma, int64_t n,
                         int32_t* __restrict__ inv, double* __restrict__ sn64, float* __restrict__ sn32) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const int32_t j = perm_n[a];
    inv[a] = off[pinv_m[j]];
    sn64[a] = sigma[j];
    sn32[a] = (float)sigma[j];
}

__global__ void k_to_f32_mf(const double* __restrict__ a, float* __restrict__ o, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) o[i] = (float)a[i];
}

inline dim3 g1d(int64_t N) { return dim3((unsigned)std::max<int64_t>(1, (N + L1LS_BLOCK - 1) / L1LS_BLOCK)); }

template <typename T>
MfTabs<T> tabs_of(const l1ls_instance* I);
template <>
MfTabs<double> tabs_of<double>(const l1ls_instance* I) {
    MfTabs<double> t;
    for (int q = 0; q < L1LS_MAX_ROUNDS; ++q) {
        t.csn[q] = I->side[0].cs[q];
        t.csm[q] = I->side[1].cs[q];
    }
    t.emb = I->mf_emb;
    t.inv = I->mf_inv;
    t.cbase = I->mf_cbase;
    t.gm = I->mfw_ws ? I->mfw_ib[0] : I->mf_emb;
    t.gn = I->mfw_ws ? I->mfw_ib[1] : I->mf_inv;
    t.xcd = I->mfw_ws ? 1 : 0;
    t.sig = I->mf_sig64;
    t.sig_n = I->mf_sign64;
    t.n = I->n;
    t.m = I->m;
    return t;
}
template <>
MfTabs<float> tabs_of<float>(const l1ls_instance* I) {
    MfTabs<float> t;
    for (int q = 0; q < L1LS_MAX_ROUNDS; ++q) {
        t.csn[q] = I->mf_cs32[0][q];
        t.csm[q] = I->mf_cs32[1][q];
    }
    t.emb = I->mf_emb;
    t.inv = I->mf_inv;
    t.cbase = I->mf_cbase;
    t.gm = I->mfw_ws ? I->mfw_ib[0] : I->mf_emb;
    t.gn = I->mfw_ws ? I->mfw_ib[1] : I->mf_inv;
    t.xcd = I->mfw_ws ? 1 : 0;
    t.sig = I->mf_sig32;
    t.sig_n = I->mf_sign32;
    t.n = I->n;
    t.m = I->m;
    return t;
}

// ---- windowed gathers -------------------------------------------------------
// A gather t -> src[idx[t]] over a vector that no cache holds costs a whole
// line per element.  The windowed form groups the targets in windows of
// 2^ws consecutive positions and the sources in chunks of 2^cs: the slots of
// a bucketed copy u are ordered by (target window, source chunk), so that
//   k_win_scatter  copies one source chunk per workgroup into u: it stages
//                  the chunk in LDS ordered by target window, then writes
//                  each (window, chunk) run of u (about 16 elements) with
//                  consecutive stores, and
//   the consumer   gathers u[ib[t]], which for the targets of a workgroup
//                  stays inside one window's segment of u, small enough to
//                  stay in L2.
// Slots within a (window, chunk) run are handed out by atomics, so the order
// of u varies between builds; every target still reads its own element, so
// the results are bitwise those of the plain gather.
constexpr int kWinMaxCs = 14;        // chunk of at most 2^14 sources: 128 KB of FP64 staging
constexpr int kWinThreads = 1024;

__global__ void k_win_count(const int32_t* __restrict__ src, int64_t NT, int ws, int cs, int64_t nc,
                            int32_t* __restrict__ cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NT) return;
    const int32_t a = src[t];
    if (a >= 0) atomicAdd(&cnt[(t >> ws) * nc + (a >> cs)], 1);
}

// cnt in (window, chunk) order -> cnt_t in (chunk, window) order
__global__ void k_win_transpose(const int32_t* __restrict__ cnt, int64_t nT, int64_t nc, int32_t* __restrict__ cnt_t) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nT * nc) return;
    const int64_t w = q / nc, c = q - w * nc;
    cnt_t[c * nT + w] = cnt[q];
}

// base: exclusive scan of the counts in (window, chunk) order (the runs of
// u); cur: a copy of it, advanced here; lbase: exclusive scan in (chunk,
// window) order (the staging order, chunk by chunk).
__global__ void k_win_assign(const int32_t* __restrict__ src, int64_t NT, int ws, int cs, int64_t nT, int64_t nc,
                             const int32_t* __restrict__ base, int32_t* __restrict__ cur,
                             const int32_t* __restrict__ lbase, int32_t* __restrict__ ib, int32_t* __restrict__ lx,
                             int32_t* __restrict__ wslot) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NT) return;
    const int32_t a = src[t];
    if (a < 0) {
        ib[t] = -1;
        return;
    }
    const int64_t w = t >> ws, c = a >> cs;
    const int32_t slot = atomicAdd(&cur[w * nc + c], 1);
    const int32_t l = lbase[c * nT + w] + (slot - base[w * nc + c]);
    ib[t] = slot;
    lx[a] = l;
    wslot[l] = slot;
}

template <typename T>
__global__ __launch_bounds__(kWinThreads) void k_win_scatter(const T* __restrict__ src, const int32_t* __restrict__ lx,
                                                              const int32_t* __restrict__ wslot, T* __restrict__ u,
                                                              int64_t N, int cs, const int32_t* __restrict__ done) {
    __shared__ T st[1 << kWinMaxCs];
    if (done && *done) return;  // the solver's converged flag (launch-uniform)
    const int64_t c0 = (int64_t)blockIdx.x << cs;
    const int cnt = (int)std::min<int64_t>((int64_t)1 << cs, N - c0);
    for (int j = threadIdx.x; j < cnt; j += kWinThreads) st[lx[c0 + j] - c0] = src[c0 + j];
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += kWinThreads) u[wslot[c0 + j]] = st[j];
}

int ceil_log2(int64_t v) {
    int r = 0;
    while (((int64_t)1 << r) < v) ++r;
    return r;
}

// Window tables of both gathers (the sources are n long on both sides).
l1ls_status build_mf_windows(l1ls_instance* I, hipStream_t s) {
    const int64_t n = I->n, m = I->m;
    const int ws = std::min(17, std::max(8, ceil_log2(n) - 6));
    DevArena tmp;
    tmp.al = I->arena.al;
    auto fail = [&](l1ls_status st) {
        (void)hipStreamSynchronize(s);
        tmp.release();
        return st;
    };
    const int32_t* srcs[2] = {I->mf_emb, I->mf_inv};
    const int64_t NT[2] = {m, n};
    for (int k = 0; k < 2; ++k) {
        const int64_t nT = (NT[k] + ((int64_t)1 << ws) - 1) >> ws;
        // about 16 sources per (window, chunk) run: a 128-byte line of FP64
        const int cs = std::min(kWinMaxCs, std::max(8, ceil_log2(nT) + 4));
        const int64_t nc = (n + ((int64_t)1 << cs) - 1) >> cs;
        if (nT * nc >= ((int64_t)1 << 31) - 1) return fail(L1LS_E_UNSUPPORTED);
        l1ls_status st;
        if ((st = I->arena.alloc(&I->mfw_ib[k], NT[k])) != L1LS_OK) return fail(st);
        if ((st = I->arena.alloc(&I->mfw_lx[k], n)) != L1LS_OK) return fail(st);
        if ((st = I->arena.alloc(&I->mfw_wslot[k], n)) != L1LS_OK) return fail(st);
        int32_t *cnt = nullptr, *cnt_t = nullptr, *base = nullptr, *cur = nullptr, *lbase = nullptr;
        const int64_t nq = nT * nc;
        if ((st = tmp.alloc(&cnt, nq)) != L1LS_OK) return fail(st);
        if ((st = tmp.alloc(&cnt_t, nq)) != L1LS_OK) return fail(st);
        if ((st = tmp.alloc(&base, nq + 1)) != L1LS_OK) return fail(st);
        if ((st = tmp.alloc(&cur, nq + 1)) != L1LS_OK) return fail(st);
        if ((st = tmp.alloc(&lbase, nq + 1)) != L1LS_OK) return fail(st);
        if (hipMemsetAsync(cnt, 0, nq * sizeof(int32_t), s) != hipSuccess) return fail(L1LS_E_HIP);
        hipLaunchKernelGGL(k_win_count, g1d(NT[k]), dim3(L1LS_BLOCK), 0, s, srcs[k], NT[k], ws, cs, nc, cnt);
        hipLaunchKernelGGL(k_win_transpose, g1d(nq), dim3(L1LS_BLOCK), 0, s, cnt, nT, nc, cnt_t);
        if ((st = exclusive_scan_i32(cnt, base, nq, s, tmp)) != L1LS_OK) return fail(st);
        if ((st = exclusive_scan_i32(cnt_t, lbase, nq, s, tmp)) != L1LS_OK) return fail(st);
        if (hipMemcpyAsync(cur, base, (nq + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
            return fail(L1LS_E_HIP);
        hipLaunchKernelGGL(k_win_assign, g1d(NT[k]), dim3(L1LS_BLOCK), 0, s, srcs[k], NT[k], ws, cs, nT, nc, base,
                           cur, lbase, I->mfw_ib[k], I->mfw_lx[k], I->mfw_wslot[k]);
        I->mfw_cs[k] = cs;
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return fail(L1LS_E_HIP);
    tmp.release();
    I->mfw_ws = ws;
    return L1LS_OK;
}

// u = the bucketed copy of the n-long source of gather k (0: w, 1: compact v)
template <typename T>
void win_scatter(const l1ls_instance* I, int k, const T* src, T* u, const int32_t* done, hipStream_t s) {
    const int cs = I->mfw_cs[k];
    const int64_t N = I->n;
    hipLaunchKernelGGL((k_win_scatter<T>), dim3((unsigned)((N + ((int64_t)1 << cs) - 1) >> cs)), dim3(kWinThreads),
                       0, s, src, I->mfw_lx[k], I->mfw_wslot[k], u, N, cs, done);
}

}  // namespace

int mf_grid(int64_t pairs);

// Lengths of the buffers a caller passes as w (n side's output) and v (the
// m side's output): with windowed gathers each also holds the bucketed copy
// at offset n.
int64_t mf_wbuf_len(const l1ls_instance* I) { return I->mfw_ws ? 2 * I->n : I->n; }
int64_t mf_vbuf_len(const l1ls_instance* I) { return I->mfw_ws ? std::max(I->m, 2 * I->n) : I->m; }

// Tables of the stage-order matrix-free operator (called by the generator).
l1ls_status build_mf_tables(l1ls_instance* I, hipStream_t s) {
    const int64_t n = I->n, m = I->m;
    L1LS_TRY(I->arena.alloc(&I->mf_emb, m));
    L1LS_TRY(I->arena.alloc(&I->mf_inv, n));
    const int64_t groups = mf_grid(m / 2);
    L1LS_TRY(I->arena.alloc(&I->mf_cbase, groups));
    L1LS_TRY(I->arena.alloc(&I->mf_sig64, m));
    L1LS_TRY(I->arena.alloc(&I->mf_sig32, m));
    L1LS_TRY(I->arena.alloc(&I->mf_sign64, n));
    L1LS_TRY(I->arena.alloc(&I->mf_sign32, n));
    L1LS_TRY(I->arena.alloc(&I->mf_b64, m));
    L1LS_TRY(I->arena.alloc(&I->mf_b32, m));
    hipLaunchKernelGGL(k_mf_emb, g1d(m), dim3(L1LS_BLOCK), 0, s, I->side[1].perm, I->side[0].pinv, I->sigma, n, m,
                       I->mf_emb, I->mf_sig64, I->mf_sig32);
    {
        // rank of the active m-positions in position order
        DevArena tmp;
        tmp.al = I->arena.al;
        int32_t *flag = nullptr, *off = nullptr;
        auto fail = [&](l1ls_status st) {
            (void)hipStreamSynchronize(s);
            tmp.release();
            return st;
        };
        l1ls_status st;
        if ((st = tmp.alloc(&flag, m)) != L1LS_OK) return fail(st);
        if ((st = tmp.alloc(&off, m + 1)) != L1LS_OK) return fail(st);
        hipLaunchKernelGGL(k_mf_active, g1d(m), dim3(L1LS_BLOCK), 0, s, I->side[1].perm, n, m, flag);
        if ((st = exclusive_scan_i32(flag, off, m, s, tmp)) != L1LS_OK) return fail(st);
        hipLaunchKernelGGL(k_mf_cbase, g1d(groups), dim3(L1LS_BLOCK), 0, s, off, m, groups, I->mf_cbase);
        hipLaunchKernelGGL(k_mf_inv, g1d(n), dim3(L1LS_BLOCK), 0, s, I->side[0].perm, I->side[1].pinv, off,
                           I->sigma, n, I->mf_inv, I->mf_sign64, I->mf_sign32);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(L1LS_E_HIP);
        tmp.release();
    }
    for (int sd = 0; sd < 2; ++sd)
        for (int t = 0; t < I->rounds; ++t) {
            const int64_t N = I->side[sd].N;
            L1LS_TRY(I->arena.alloc(&I->mf_cs32[sd][t], N));
            hipLaunchKernelGGL(k_to_f32_mf, g1d(N), dim3(L1LS_BLOCK), 0, s, I->side[sd].cs[t], I->mf_cs32[sd][t], N);
        }
    hipLaunchKernelGGL((k_gather_perm<double, double>), g1d(m), dim3(L1LS_BLOCK), 0, s, I->b, I->mf_b64,
                       I->side[1].perm, m);
    hipLaunchKernelGGL((k_gather_perm<float, double>), g1d(m), dim3(L1LS_BLOCK), 0, s, I->b, I->mf_b32,
                       I->side[1].perm, m);
    HIP_TRY(hipGetLastError());
    // windowed gathers once the gathered vectors (n entries) outgrow the
    // caches: measured slower at n = 2^20, faster from n = 2^22 on
    if ((I->storage & L1LS_STORE_MF_WINDOWS) || n >= ((int64_t)1 << 22)) L1LS_TRY(build_mf_windows(I, s));
    return L1LS_OK;
}

// Grid of the matrix-free passes: one thread per rotation pair, one
// workgroup per 256 pairs.
int mf_grid(int64_t pairs) { return (int)std::max<int64_t>(1, (pairs + L1LS_BLOCK - 1) / L1LS_BLOCK); }

// w has n entries (n order), vt has m entries (m order).
// Residual pass: on the first pass (init) w = Sigma_n G^T x is formed first;
// afterwards it comes from the preceding transpose pass.  vt (m entries)
// receives Sigma_m Q^T r_y for the next transpose pass; w has n entries.
template <typename T>
void mf_residual_launch(const l1ls_instance* I, const T* x, T* w, const T* b, const T* rx_prev, T* rx, T* vt,
                        T beta, int init, double* part, const GapState* gs, int stats, hipStream_t s) {
    const MfTabs<T> tb = tabs_of<T>(I);
    const int32_t* done = gs ? &gs->done : nullptr;
    if (init) {
        if (I->rounds == 2)
            hipLaunchKernelGGL((k_mf_gt<T, 2>), dim3(mf_grid(I->n / 2)), dim3(L1LS_BLOCK), 0, s, x, w, tb, done);
        else
            hipLaunchKernelGGL((k_mf_gt<T, 1>), dim3(mf_grid(I->n / 2)), dim3(L1LS_BLOCK), 0, s, x, w, tb, done);
    }
    const T* wg = w;  // what the m side gathers from
    if (I->mfw_ws) {
        win_scatter<T>(I, 0, w, w + I->n, done, s);
        wg = w + I->n;
    }
    if (I->rounds == 2)
        hipLaunchKernelGGL((k_mf_res_qt<T, 2>), dim3(mf_grid(I->m / 2)), dim3(L1LS_BLOCK), 0, s, wg, b, rx_prev, rx,
                           vt, beta, init, tb, part, done, stats);
    else
        hipLaunchKernelGGL((k_mf_res_qt<T, 1>), dim3(mf_grid(I->m / 2)), dim3(L1LS_BLOCK), 0, s, wg, b, rx_prev, rx,
                           vt, beta, init, tb, part, done, stats);
}

// Transpose pass (with prox) from vt; also forms w = Sigma_n G^T x_k for the
// residual pass that follows.
template <typename T>
void mf_transpose_launch(const l1ls_instance* I, T* vt, T* w, const T* xc, const T* xp, T* xo, T beta, T L,
                         T thr, double* part, const GapState* gs, int stats, hipStream_t s) {
    const MfTabs<T> tb = tabs_of<T>(I);
    const T* vg = vt;  // what the n side gathers from
    if (I->mfw_ws) {
        win_scatter<T>(I, 1, vt, vt + I->n, gs ? &gs->done : nullptr, s);
        vg = vt + I->n;
    }
    if (I->rounds == 2)
        hipLaunchKernelGGL((k_mf_prox_gt<T, 2>), dim3(mf_grid(I->n / 2)), dim3(L1LS_BLOCK), 0, s, vg, xc, xp, xo,
                           w, beta, L, thr, tb, part, gs, stats);
    else
        hipLaunchKernelGGL((k_mf_prox_gt<T, 1>), dim3(mf_grid(I->n / 2)), dim3(L1LS_BLOCK), 0, s, vg, xc, xp, xo,
                           w, beta, L, thr, tb, part, gs, stats);
}

template void mf_residual_launch<float>(const l1ls_instance*, const float*, float*, const float*, const float*,
                                        float*, float*, float, int, double*, const GapState*, int, hipStream_t);
template void mf_residual_launch<double>(const l1ls_instance*, const double*, double*, const double*,
                                         const double*, double*, double*, double, int, double*, const GapState*, int,
                                         hipStream_t);
template void mf_transpose_launch<float>(const l1ls_instance*, float*, float*, const float*, const float*,
                                         float*, float, float, float, double*, const GapState*, int, hipStream_t);
template void mf_transpose_launch<double>(const l1ls_instance*, double*, double*, const double*,
                                          const double*, double*, double, double, double, double*, const GapState*,
                                          int, hipStream_t);

// ---- products for the second-order path (FP64, stage order) -----------------
// A x with x (n) and out (m) in stage order: w = Sigma_n G^T x, then the
// m-side pass writes out = A x.
// TT: type of the rotation tables and sigma (double, or float for the
// FP32-coefficient Hessian products); vectors and arithmetic are FP64.
template <int MODE, typename TT>
void mf_fwd_launch(const l1ls_instance* I, const double* x, double* wn, double* out, double* vm, const int32_t* done,
                   hipStream_t s) {
    const MfTabs<TT> tb = tabs_of<TT>(I);
    if (I->rounds == 2)
        hipLaunchKernelGGL((k_mf_gt<double, 2, TT>), dim3(mf_grid(I->n / 2)), dim3(L1LS_BLOCK), 0, s, x, wn, tb,
                           done);
    else
        hipLaunchKernelGGL((k_mf_gt<double, 1, TT>), dim3(mf_grid(I->n / 2)), dim3(L1LS_BLOCK), 0, s, x, wn, tb,
                           done);
    const double* wg = wn;
    if (I->mfw_ws) {
        win_scatter<double>(I, 0, wn, wn + I->n, done, s);
        wg = wn + I->n;
    }
    if (I->rounds == 2)
        hipLaunchKernelGGL((k_mf_res_qt<double, 2, MODE, TT>), dim3(mf_grid(I->m / 2)), dim3(L1LS_BLOCK), 0, s, wg,
                           (const double*)nullptr, (const double*)nullptr, out, vm, 0.0, 1, tb, (double*)nullptr,
                           done, 0);
    else
        hipLaunchKernelGGL((k_mf_res_qt<double, 1, MODE, TT>), dim3(mf_grid(I->m / 2)), dim3(L1LS_BLOCK), 0, s, wg,
                           (const double*)nullptr, (const double*)nullptr, out, vm, 0.0, 1, tb, (double*)nullptr,
                           done, 0);
}

void mf_apply_fwd(const l1ls_instance* I, const double* x, double* wn, double* out, hipStream_t s) {
    mf_fwd_launch<kMfProduct, double>(I, x, wn, out, (double*)nullptr, (const int32_t*)nullptr, s);
}

// out (n) = A^T y with y (m) and out in stage order; vm is scratch of
// mf_vbuf_len entries.
void mf_apply_adj(const l1ls_instance* I, const double* y, double* vm, double* out, hipStream_t s) {
    const MfTabs<double> tb = tabs_of<double>(I);
    if (I->rounds == 2)
        hipLaunchKernelGGL((k_mf_qt<double, 2>), dim3(mf_grid(I->m / 2)), dim3(L1LS_BLOCK), 0, s, y, vm, tb);
    else
        hipLaunchKernelGGL((k_mf_qt<double, 1>), dim3(mf_grid(I->m / 2)), dim3(L1LS_BLOCK), 0, s, y, vm, tb);
    const double* vg = vm;
    if (I->mfw_ws) {
        win_scatter<double>(I, 1, vm, vm + I->n, (const int32_t*)nullptr, s);
        vg = vm + I->n;
    }
    if (I->rounds == 2)
        hipLaunchKernelGGL((k_mf_g_hess<double, 2>), dim3(mf_grid(I->n / 2)), dim3(L1LS_BLOCK), 0, s, vg,
                           (const double*)nullptr, (const double*)nullptr, (const uint8_t*)nullptr, out, tb,
                           (double*)nullptr, (const int32_t*)nullptr);
    else
        hipLaunchKernelGGL((k_mf_g_hess<double, 1>), dim3(mf_grid(I->n / 2)), dim3(L1LS_BLOCK), 0, s, vg,
                           (const double*)nullptr, (const double*)nullptr, (const uint8_t*)nullptr, out, tb,
                           (double*)nullptr, (const int32_t*)nullptr);
}

// hp = mask (A^T A p + d p) with part[block] = sum p hp over mf_grid(n/2)
// blocks (A p itself is not stored).  Skipped once *done is set.
template <typename TT>
void mf_hess_t(const l1ls_instance* I, const double* p, double* wn, double* vm, const double* d,
               const uint8_t* mask, double* hp, double* part, const int32_t* done, hipStream_t s) {
    mf_fwd_launch<kMfNormal, TT>(I, p, wn, (double*)nullptr, vm, done, s);
    const MfTabs<TT> tb = tabs_of<TT>(I);
    const double* vg = vm;
    if (I->mfw_ws) {
        win_scatter<double>(I, 1, vm, vm + I->n, done, s);
        vg = vm + I->n;
    }
    if (I->rounds == 2)
        hipLaunchKernelGGL((k_mf_g_hess<double, 2, TT>), dim3(mf_grid(I->n / 2)), dim3(L1LS_BLOCK), 0, s, vg, p, d,
                           mask, hp, tb, part, done);
    else
        hipLaunchKernelGGL((k_mf_g_hess<double, 1, TT>), dim3(mf_grid(I->n / 2)), dim3(L1LS_BLOCK), 0, s, vg, p, d,
                           mask, hp, tb, part, done);
}

// f32: the rotation coefficients and sigma of the products are the FP32
// copies (vectors and sums stay FP64), as the stored path's FP32 values.
void mf_hess(const l1ls_instance* I, const double* p, double* wn, double* vm, const double* d, const uint8_t* mask,
             double* hp, double* part, const int32_t* done, hipStream_t s, bool f32) {
    if (f32)
        mf_hess_t<float>(I, p, wn, vm, d, mask, hp, part, done, s);
    else
        mf_hess_t<double>(I, p, wn, vm, d, mask, hp, part, done, s);
}
