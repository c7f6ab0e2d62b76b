// The A = Sigma G^T instance class of sections 8.4 to 8.9 (Table 1), its
// CG-Newton and its FISTA.
//
// The experiments of sections 8.4, 8.5, 8.6 and 8.9 use A = Sigma G^T with
// m >= n rows (m = 2n there) and rank n: Sigma carries sigma_1..sigma_n on
// its top n x n diagonal (section 4, the display of Sigma), and G is one
// stage of n/2 Givens rotations G(2k-1, 2k, theta) on adjacent pairs with one
// shared angle (section 4.1 with Q = I and no permutation).  The singular
// values alternate between two values (section 8.9) or are uniform on
// [0, 10^q] shifted by 0.1 (sections 8.4 to 8.6); x* is Table 1's
// (section 8.9), Procedure OsGen's or Procedure OsGen3's (section 6); b comes
// from Procedure IGen (section 3.1).
//
// Every row and column of A couples the two elements of one pair and rows
// n..m-1 are zero, so A is block diagonal with one 2 x 2 block per pair.
// Nothing is gathered: a thread owns whole pairs, reads each vector as one
// 16-byte double2 per pair, and every product with A, A^T, A^T A and the
// Hessian of (8) is formed in registers.  The instance stores b only (its
// top n entries; the others are zero); sigma, x* and the subgradient g are
// pure functions of (seed, index) and, for OsGen3, of two selection
// thresholds kept in the instance, recomputed wherever they are needed.
//
// CG-Newton follows section 8.1 (item pdNCG) and section 8.3 exactly as the
// stored-operator solver does: smoothed problem (8) with the pseudo-Huber
// function (7), Newton directions from PCG with the inverse Hessian diagonal
// as preconditioner, Armijo backtracking by halving.  PCG runs in the
// single-reduction form of Chronopoulos and Gear (J. Comput. Appl. Math. 25,
// 1989): the preconditioned residual u = M r, w = H u and s = H p are
// products with the block-diagonal Hessian, formed in registers from r, p
// and the Hessian diagonal d, so one PCG iteration is one streaming pass
// (read r, d, p, dx; write p, dx, r: 56 bytes per variable) and one
// reduction of (r.u, w.u, r.r).  In exact arithmetic its iterates are those
// of the textbook recurrence the oracle runs.  FISTA (section 8.1) is one
// pass per iteration (read x_k, x_{k-1}, b; write x_{k+1}: 32 bytes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "rng.hpp"

using namespace l1ls;

namespace {

constexpr int kHB = 256;            // threads per block of the streaming kernels
constexpr int kHMaxBlocks = 16384;  // grid cap (64 blocks per CU); partial sums per block
constexpr int kHU = 2;              // pairs per thread per trip of the PCG pass
constexpr bool kHNT = true;         // nontemporal loads and stores in the PCG pass
constexpr int kLsBatch = 8;        // step lengths tried per line-search pass
constexpr int kLsStats = 3 + 2 * kLsBatch;
constexpr int64_t kSgtMaxN = (int64_t)1 << 32;  // Philox counter word 0 holds the index
constexpr uint32_t kTagSigma = 0x500u;          // uniform singular values, per pair
constexpr int kSelBins = 256;                   // radix-select digit of 8 bits

// Constants of one instance, passed by value to every kernel.
struct SgtK {
    int64_t n, s, s1, s2;
    int64_t np;       // row pairs with entries: min(m, n) / 2
    int64_t nnp;      // IGen2 (m < n): column pairs of N~, in the rows of pairs k < nnp; else 0
    int64_t noff;     // IGen2: pair index in x of N~'s first column pair (m / 2)
    int64_t nsup;     // range of supp(x*): n, or m for IGen2
    const double* cs; // IGen2: column scales xi_j tau / |N_j^T e| of N~ (n - m)
    int32_t sigma_law, xstar_law;
    double c, sn;              // cos, sin of the shared angle
    double so, se;             // alternating law: sigma at the first / second element of a pair
    double cn0, cn1;           // alternating law: diag(A^T A) at the first / second element
    double scale, shift;       // uniform law: sigma = u * scale + shift
    double tau, xneg, xpos, gamma;
    // OsGen3: the kept components are those at or below (t1_bits, t1_idx) and at
    // or above (t2_bits, t2_idx) in the order (|x_i|, i); has1 / has2 = 0: none
    uint64_t t1_bits, t2_bits;
    int64_t t1_idx, t2_idx;
    int32_t has1, has2;
    Key key;
};

struct HCg {
    double gamma, rr0, stop, alpha, beta, gmax;
    int32_t iters, done;
};

// 16-byte vector type the nontemporal builtins accept
typedef double dv2 __attribute__((ext_vector_type(2)));

// Uniform law: Philox counter (k, 0, kTagSigma, 0), words (0, 1) for the
// first element and (2, 3) for the second, each u * scale + shift with the
// product and the sum rounded separately (no fused multiply-add).
__device__ __forceinline__ double2 uniform_sigma_pair(const SgtK& H, int64_t k) {
#pragma clang fp contract(off)
    const U4 w = philox4x32_10((uint32_t)k, 0u, kTagSigma, 0u, H.key.k0, H.key.k1);
    return make_double2(unit_double(w.x, w.y) * H.scale + H.shift, unit_double(w.z, w.w) * H.scale + H.shift);
}

// sigma of pair k (elements 2k, 2k+1)
template <int SL>
__device__ __forceinline__ double2 sigma_pair(const SgtK& H, int64_t k) {
    if constexpr (SL == 0)
        return make_double2(H.so, H.se);
    else
        return uniform_sigma_pair(H, k);
}

// diag(A^T A) on the pair: squared norms of the two columns of the block
template <int SL>
__device__ __forceinline__ double2 colnorm_pair(const SgtK& H, double2 sg) {
    if constexpr (SL == 0) {
        return make_double2(H.cn0, H.cn1);
    } else {
        const double a = sg.x * sg.x, b = sg.y * sg.y, c2 = H.c * H.c, s2 = H.sn * H.sn;
        return make_double2(a * c2 + b * s2, a * s2 + b * c2);
    }
}

// (y_i, y_j) = block of A x: sigma (G^T x) on the pair
__device__ __forceinline__ void a_pair(const SgtK& H, double2 sg, double xi, double xj, double& yi, double& yj) {
    yi = sg.x * (H.c * xi + H.sn * xj);
    yj = sg.y * (-H.sn * xi + H.c * xj);
}

// (x_i, x_j) = block of A^T y: G (sigma y) on the pair
__device__ __forceinline__ void at_pair(const SgtK& H, double2 sg, double yi, double yj, double& xi, double& xj) {
    const double ti = sg.x * yi, tj = sg.y * yj;
    xi = H.c * ti - H.sn * tj;
    xj = H.sn * ti + H.c * tj;
}

// H p = A^T (A p) + d p on the pair
__device__ __forceinline__ double2 hess_pair(const SgtK& H, double2 sg, double2 p, double2 d) {
    double yi, yj, hi, hj;
    a_pair(H, sg, p.x, p.y, yi, yj);
    at_pair(H, sg, yi, yj, hi, hj);
    return make_double2(hi + d.x * p.x, hj + d.y * p.y);
}

// IGen2: sigma of N's column pair k; uniform law from counter (k, 1, kTagSigma, 0)
__device__ __forceinline__ double2 uniform_sigma_n_pair(const SgtK& H, int64_t k) {
#pragma clang fp contract(off)
    const U4 w = philox4x32_10((uint32_t)k, 1u, kTagSigma, 0u, H.key.k0, H.key.k1);
    return make_double2(unit_double(w.x, w.y) * H.scale + H.shift, unit_double(w.z, w.w) * H.scale + H.shift);
}

template <int SL>
__device__ __forceinline__ double2 sigma_n_pair(const SgtK& H, int64_t k) {
    if constexpr (SL == 0)
        return make_double2(H.so, H.se);
    else
        return uniform_sigma_n_pair(H, k);
}

// Row pair k: B's block (sigma sb) and, for IGen2 rows k < nnp, N~'s block
// (sigma sn, column scales cs).  NN = 0 compiles the m >= n class alone.
struct Row {
    double2 sb, sn, cs;
    bool hasN;
};

template <int SL, int NN>
__device__ __forceinline__ Row load_row(const SgtK& H, int64_t k) {
    Row R;
    R.sb = sigma_pair<SL>(H, k);
    R.hasN = NN && k < H.nnp;
    if (NN && R.hasN) {
        R.sn = sigma_n_pair<SL>(H, k);
        R.cs = reinterpret_cast<const double2*>(H.cs)[k];
    } else {
        R.sn = make_double2(0.0, 0.0);
        R.cs = make_double2(0.0, 0.0);
    }
    return R;
}

// rows of the pair: B x_B + N~ x_N (N~ = N diag(cs))
template <int NN>
__device__ __forceinline__ void a_row(const SgtK& H, const Row& R, double2 xb, double2 xn, double& yi, double& yj) {
    a_pair(H, R.sb, xb.x, xb.y, yi, yj);
    if (NN && R.hasN) {
        double ui, uj;
        a_pair(H, R.sn, R.cs.x * xn.x, R.cs.y * xn.y, ui, uj);
        yi += ui;
        yj += uj;
    }
}

// columns of the pair: g_B = B^T r, g_N = N~^T r
template <int NN>
__device__ __forceinline__ void at_row(const SgtK& H, const Row& R, double ri, double rj, double2& gb, double2& gn) {
    at_pair(H, R.sb, ri, rj, gb.x, gb.y);
    gn = make_double2(0.0, 0.0);
    if (NN && R.hasN) {
        double ti, tj;
        at_pair(H, R.sn, ri, rj, ti, tj);
        gn = make_double2(R.cs.x * ti, R.cs.y * tj);
    }
}

// diag(A^T A) on B's and N~'s column pairs
template <int SL, int NN>
__device__ __forceinline__ void colnorm_row(const SgtK& H, const Row& R, double2& cb, double2& cn) {
    cb = colnorm_pair<SL>(H, R.sb);
    cn = make_double2(0.0, 0.0);
    if (NN && R.hasN) {
        const double2 c0 = colnorm_pair<SL>(H, R.sn);
        cn = make_double2(R.cs.x * R.cs.x * c0.x, R.cs.y * R.cs.y * c0.y);
    }
}

// OsGen3 before selection: x = G gamma (Sigma^T Sigma)^{-1} 1_n on the pair,
// the exact minimiser of eq. (19), in the operation order of the definition.
__device__ __forceinline__ double2 osgen3_full_pair(const SgtK& H, double2 sg) {
#pragma clang fp contract(off)
    const double vi = H.gamma / (sg.x * sg.x), vj = H.gamma / (sg.y * sg.y);
    return make_double2(H.c * vi - H.sn * vj, H.sn * vi + H.c * vj);
}

__device__ __forceinline__ uint64_t abs_bits(double v) { return (uint64_t)__double_as_longlong(fabs(v)); }

// (a, i) <= (b, j) in the order by magnitude, then index
__device__ __forceinline__ bool key_le(uint64_t a, int64_t i, uint64_t b, int64_t j) {
    return a < b || (a == b && i <= j);
}

// x*_i and the subgradient g_i of IGen step 2 for element i with the value
// xf (OsGen3's unselected x) of its pair.  Table 1 and OsGen: i is in
// supp(x*) when its position q under the inverse support bijection is < s
// (the support is the first s outputs of that bijection); off the support
// g_i = 0.9 (2u - 1).
__device__ __forceinline__ void planted_elem(const SgtK& H, int64_t i, double xf, double& xs, double& g) {
    bool on = false;
    xs = 0.0;
    if (H.xstar_law == L1LS_XSTAR_OSGEN3) {
        const uint64_t kb = abs_bits(xf);
        on = (H.has1 && key_le(kb, i, H.t1_bits, H.t1_idx)) || (H.has2 && key_le(H.t2_bits, H.t2_idx, kb, i));
        if (on) xs = xf;
    } else if (H.s > 0) {
        const int64_t q = bijection_inverse(i, H.nsup, kTagPerm | 2u, H.key);
        if (q < H.s) {
            on = true;
            if (H.xstar_law == L1LS_XSTAR_TABLE1) {
                xs = (q < H.s / 2) ? H.xneg : H.xpos;
            } else {
                const U4 w = philox4x32_10((uint32_t)q, 0u, kTagXstar, 0u, H.key.k0, H.key.k1);
                xs = H.gamma * (2.0 * unit_double(w.x, w.y) - 1.0);  // 2u is exact: a fused form rounds the same
            }
        }
    }
    if (on) {
        g = xs > 0.0 ? 1.0 : (xs < 0.0 ? -1.0 : 0.0);
    } else {
        const U4 w = philox4x32_10((uint32_t)i, 0u, kTagSubgrad, 0u, H.key.k0, H.key.k1);
        g = 0.9 * (2.0 * unit_double(w.x, w.y) - 1.0);  // 2u is exact: a fused form rounds the same
    }
}

// x* and g on pair k with singular values sg
__device__ __forceinline__ void planted_pair(const SgtK& H, int64_t k, double2 sg, double2& xs, double2& g) {
    double2 xf = make_double2(0.0, 0.0);
    if (H.xstar_law == L1LS_XSTAR_OSGEN3) xf = osgen3_full_pair(H, sg);
    planted_elem(H, 2 * k, xf.x, xs.x, g.x);
    planted_elem(H, 2 * k + 1, xf.y, xs.y, g.y);
}

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

template <int NS, int NSUM>
__device__ __forceinline__ void store_partials(double (&v)[NS], double* __restrict__ part) {
    block_reduce_stats<NS, NSUM>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NS; ++q) part[(size_t)NS * blockIdx.x + q] = v[q];
    }
}

// ---- instance ----------------------------------------------------------------
// IGen steps 3 and 4 on one pair: e = tau Sigma^{-1} G^T g and b = A x* + e,
// each operation rounded on its own (no fused multiply-add), in the order
// the definition writes them.
__device__ __forceinline__ void igen_pair(const SgtK& H, double2 sg, double2 xs, double2 g, double2& b,
                                          double2& e) {
#pragma clang fp contract(off)
    e.x = H.tau * (H.c * g.x + H.sn * g.y) / sg.x;
    e.y = H.tau * (-H.sn * g.x + H.c * g.y) / sg.y;
    b.x = sg.x * (H.c * xs.x + H.sn * xs.y) + e.x;
    b.y = sg.y * (-H.sn * xs.x + H.c * xs.y) + e.y;
}

// b for every row pair, and for IGen2 the column scales of N~ (IGen2 step 4:
// N~_j = xi_j tau / |N_j^T e| N_j, xi_j = 2u - 1 from counter (j, 0, kTagXi, 0));
// part = (sum e^2, sum |x*| | max sigma, max -sigma, max row eigenvalue of A A^T)
constexpr uint32_t kTagXi = 0x700u;

__device__ __forceinline__ double2 igen2_scales(const SgtK& H, int64_t k, double2 sn, double2 e) {
#pragma clang fp contract(off)
    const double ti = sn.x * e.x, tj = sn.y * e.y;
    const double ni = H.c * ti - H.sn * tj, nj = H.sn * ti + H.c * tj;  // N^T e on the pair
    const U4 wi = philox4x32_10((uint32_t)(2 * k), 0u, kTagXi, 0u, H.key.k0, H.key.k1);
    const U4 wj = philox4x32_10((uint32_t)(2 * k + 1), 0u, kTagXi, 0u, H.key.k0, H.key.k1);
    const double xi = 2.0 * unit_double(wi.x, wi.y) - 1.0, xj = 2.0 * unit_double(wj.x, wj.y) - 1.0;
    return make_double2(xi * H.tau / fabs(ni), xj * H.tau / fabs(nj));
}

template <int SL, int NN>
__global__ __launch_bounds__(kHB) void kh_generate(SgtK H, double2* __restrict__ b, double2* __restrict__ csw,
                                                   double* __restrict__ part) {
    double v[5] = {0.0, 0.0, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = gtid(); k < H.np; k += gstride()) {
        const double2 sg = sigma_pair<SL>(H, k);
        double2 xs, g, bv, e;
        planted_pair(H, k, sg, xs, g);
        igen_pair(H, sg, xs, g, bv, e);
        b[k] = bv;
        v[0] += e.x * e.x + e.y * e.y;
        v[1] += fabs(xs.x) + fabs(xs.y);
        v[2] = fmax(v[2], fmax(sg.x, sg.y));
        v[3] = fmax(v[3], fmax(-sg.x, -sg.y));
        double lam = fmax(sg.x * sg.x, sg.y * sg.y);
        if (NN && k < H.nnp) {
            const double2 sn = sigma_n_pair<SL>(H, k);
            const double2 cs = igen2_scales(H, k, sn, e);
            csw[k] = cs;
            // rows of [B, N~] on the pair and the larger eigenvalue of their Gram matrix
            const double bi0 = sg.x * H.c, bi1 = sg.x * H.sn, bj0 = -sg.y * H.sn, bj1 = sg.y * H.c;
            const double ni0 = sn.x * H.c * cs.x, ni1 = sn.x * H.sn * cs.y;
            const double nj0 = -sn.y * H.sn * cs.x, nj1 = sn.y * H.c * cs.y;
            const double a11 = bi0 * bi0 + bi1 * bi1 + ni0 * ni0 + ni1 * ni1;
            const double a22 = bj0 * bj0 + bj1 * bj1 + nj0 * nj0 + nj1 * nj1;
            const double a12 = bi0 * bj0 + bi1 * bj1 + ni0 * nj0 + ni1 * nj1;
            const double h = 0.5 * (a11 - a22);
            lam = 0.5 * (a11 + a22) + sqrt(h * h + a12 * a12);
        }
        v[4] = fmax(v[4], lam);
    }
    store_partials<5, 2>(v, part);
}

// x* and g (n each; IGen2: entries m..n-1 are 0, g being defined on the first m)
template <int SL, int NN>
__global__ __launch_bounds__(kHB) void kh_planted(SgtK H, double* __restrict__ xs, double* __restrict__ g) {
    for (int64_t k = gtid(); k < H.np; k += gstride()) {
        double2 a, c;
        planted_pair(H, k, sigma_pair<SL>(H, k), a, c);
        if (xs) {
            xs[2 * k] = a.x;
            xs[2 * k + 1] = a.y;
        }
        if (g) {
            g[2 * k] = c.x;
            g[2 * k + 1] = c.y;
        }
        if (NN && k < H.nnp) {
            const int64_t j = 2 * (H.noff + k);
            if (xs) xs[j] = xs[j + 1] = 0.0;
            if (g) g[j] = g[j + 1] = 0.0;
        }
    }
}

// part = (sum (x - x*)^2, sum x*^2)
template <int SL, int NN>
__global__ __launch_bounds__(kHB) void kh_err(SgtK H, const double2* __restrict__ x, double* __restrict__ part) {
    double v[2] = {0.0, 0.0};
    for (int64_t k = gtid(); k < H.np; k += gstride()) {
        double2 a, c;
        planted_pair(H, k, sigma_pair<SL>(H, k), a, c);
        const double2 xv = x[k];
        const double di = xv.x - a.x, dj = xv.y - a.y;
        v[0] += di * di + dj * dj;
        v[1] += a.x * a.x + a.y * a.y;
        if (NN && k < H.nnp) {
            const double2 xn = x[H.noff + k];  // x*_N = 0
            v[0] += xn.x * xn.x + xn.y * xn.y;
        }
    }
    store_partials<2, 2>(v, part);
}

// kappa_rho of eq. (17) at x = x*: the eigenvectors of A^T A = G Sigma^2 G^T
// are the columns of G with eigenvalues sigma_i^2, so ||P_rho x||^2 sums
// (G^T x)_i^2 over sigma_i^2 >= rho.  part = (sum x^2, sum (G^T x)_i^2 [sigma_i^2 >= rho])
template <int SL>
__global__ __launch_bounds__(kHB) void kh_kappa(SgtK H, double rho, double* __restrict__ part) {
    double v[2] = {0.0, 0.0};
    const int64_t np = H.n / 2;
    for (int64_t k = gtid(); k < np; k += gstride()) {
        const double2 sg = sigma_pair<SL>(H, k);
        double2 a, c;
        planted_pair(H, k, sg, a, c);
        const double ui = H.c * a.x + H.sn * a.y, uj = -H.sn * a.x + H.c * a.y;
        v[0] += a.x * a.x + a.y * a.y;
        if (sg.x * sg.x >= rho) v[1] += ui * ui;
        if (sg.y * sg.y >= rho) v[1] += uj * uj;
    }
    store_partials<2, 2>(v, part);
}

// One radix-select pass over the OsGen3 keys (|x_i| bits, i) before
// selection.  by_index = 0: count the digit (bits >> shift) & 255 of the
// elements whose bits match `prefix` under `mask`; by_index = 1: count the
// digit (i >> shift) & 255 of the elements with bits == value whose index
// matches prefix under mask.  Block histograms in LDS, then added to hist.
template <int SL>
__global__ __launch_bounds__(kHB) void kh_select_hist(SgtK H, int by_index, uint64_t value, uint64_t prefix,
                                                      uint64_t mask, int shift,
                                                      unsigned long long* __restrict__ hist) {
    __shared__ uint32_t lh[kSelBins];
    for (int q = threadIdx.x; q < kSelBins; q += blockDim.x) lh[q] = 0u;
    __syncthreads();
    const int64_t np = H.n / 2;
    for (int64_t k = gtid(); k < np; k += gstride()) {
        const double2 xf = osgen3_full_pair(H, sigma_pair<SL>(H, k));
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const uint64_t kb = abs_bits(e ? xf.y : xf.x);
            const uint64_t idx = (uint64_t)(2 * k + e);
            if (!by_index) {
                if ((kb & mask) == prefix) atomicAdd(&lh[(kb >> shift) & 255u], 1u);
            } else if (kb == value && (idx & mask) == prefix) {
                atomicAdd(&lh[(idx >> shift) & 255u], 1u);
            }
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kSelBins; q += blockDim.x)
        if (lh[q]) atomicAdd(&hist[q], (unsigned long long)lh[q]);
}

// trans = 0: out (m) = A in (n), rows beyond the row pairs zero; trans = 1:
// out (n) = A^T in (m)
template <int SL, int NN>
__global__ __launch_bounds__(kHB) void kh_apply(SgtK H, int64_t m, int trans, const double2* __restrict__ in,
                                                double2* __restrict__ out) {
    const int64_t total = trans ? H.np : m / 2;
    for (int64_t k = gtid(); k < total; k += gstride()) {
        if (k >= H.np) {
            out[k] = make_double2(0.0, 0.0);
            continue;
        }
        const Row R = load_row<SL, NN>(H, k);
        if (trans) {
            const double2 a = in[k];
            double2 gb, gn;
            at_row<NN>(H, R, a.x, a.y, gb, gn);
            out[k] = gb;
            if (NN && R.hasN) out[H.noff + k] = gn;
        } else {
            const double2 xb = in[k];
            const double2 xn = (NN && R.hasN) ? in[H.noff + k] : make_double2(0.0, 0.0);
            double yi, yj;
            a_row<NN>(H, R, xb, xn, yi, yj);
            out[k] = make_double2(yi, yj);
        }
    }
}

// part = (sum |x|, sum r^2, sum b r | max |A^T r|), r = A x - b
template <int SL, int NN>
__global__ __launch_bounds__(kHB) void kh_gap(SgtK H, const double2* __restrict__ x, const double2* __restrict__ b,
                                              double* __restrict__ part) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t k = gtid(); k < H.np; k += gstride()) {
        const Row R = load_row<SL, NN>(H, k);
        const double2 xv = x[k], bv = b[k];
        const double2 xn = (NN && R.hasN) ? x[H.noff + k] : make_double2(0.0, 0.0);
        double yi, yj;
        a_row<NN>(H, R, xv, xn, yi, yj);
        const double ri = yi - bv.x, rj = yj - bv.y;
        double2 gb, gn;
        at_row<NN>(H, R, ri, rj, gb, gn);
        v[0] += fabs(xv.x) + fabs(xv.y) + fabs(xn.x) + fabs(xn.y);
        v[1] += ri * ri + rj * rj;
        v[2] += bv.x * ri + bv.y * rj;
        v[3] = fmax(v[3], fmax(fmax(fabs(gb.x), fabs(gb.y)), fmax(fabs(gn.x), fabs(gn.y))));
    }
    store_partials<4, 3>(v, part);
}

// ---- FISTA -------------------------------------------------------------------
// Iteration k of section 8.1's FISTA on a row pair: y = x_{k-1} + beta
// (x_{k-1} - x_{k-2}), x_k = soft(y - A^T (A y - b) / L, tau / L).  xc holds
// x_{k-1}; xo holds x_{k-2} on entry and x_k on exit.
template <int SL, int NN>
__global__ __launch_bounds__(kHB) void kh_fista(SgtK H, const dv2* __restrict__ xc, dv2* __restrict__ xo,
                                                const dv2* __restrict__ b, double beta, double L, double thr) {
    for (int64_t k = gtid(); k < H.np; k += gstride()) {
        const Row R = load_row<SL, NN>(H, k);
        const dv2 xv = __builtin_nontemporal_load(xc + k), xp = __builtin_nontemporal_load(xo + k);
        const dv2 bv = __builtin_nontemporal_load(b + k);
        const dv2 y = xv + beta * (xv - xp);
        dv2 yn = {0.0, 0.0};
        if (NN && R.hasN) {
            const dv2 xvn = xc[H.noff + k], xpn = xo[H.noff + k];
            yn = xvn + beta * (xvn - xpn);
        }
        double ri, rj;
        a_row<NN>(H, R, make_double2(y.x, y.y), make_double2(yn.x, yn.y), ri, rj);
        double2 gb, gn;
        at_row<NN>(H, R, ri - bv.x, rj - bv.y, gb, gn);
        dv2 xn;
        xn.x = soft_threshold<double>(y.x - gb.x / L, thr);
        xn.y = soft_threshold<double>(y.y - gb.y / L, thr);
        __builtin_nontemporal_store(xn, xo + k);
        if (NN && R.hasN) {
            dv2 xnn;
            xnn.x = soft_threshold<double>(yn.x - gn.x / L, thr);
            xnn.y = soft_threshold<double>(yn.y - gn.y / L, thr);
            xo[H.noff + k] = xnn;
        }
    }
}

// ---- PCDM ----------------------------------------------------------------------
// One synchronous step of section 8.1's PCDM on a row pair: from the same x,
// every sampled coordinate i takes x_i <- soft(x_i - A_i^T (A x - b) / v_i,
// tau / v_i) with v_i = beta L_i, L_i = (A^T A)_ii.  The coordinates of the
// pair at index q of x (q = k for B's pair, noff + k for N~'s) are sampled
// when words 0 and 1 of Philox counter (q, step, kTagPcdm, 0) are below thr
// (every coordinate when thr = 2^32).  x is updated in place.
constexpr uint32_t kTagPcdm = 0x600u;

__device__ __forceinline__ dv2 pcdm_pick(const SgtK& H, int64_t q, uint32_t step, uint64_t thr, dv2 upd, dv2 old) {
    if (thr < ((uint64_t)1 << 32)) {
        const U4 w = philox4x32_10((uint32_t)q, step, kTagPcdm, 0u, H.key.k0, H.key.k1);
        if (!((uint64_t)w.x < thr)) upd.x = old.x;
        if (!((uint64_t)w.y < thr)) upd.y = old.y;
    }
    return upd;
}

template <int SL, int NN>
__global__ __launch_bounds__(kHB) void kh_pcdm(SgtK H, dv2* __restrict__ x, const dv2* __restrict__ b, double beta,
                                               uint64_t thr, uint32_t step) {
    for (int64_t k = gtid(); k < H.np; k += gstride()) {
        const Row R = load_row<SL, NN>(H, k);
        double2 cb, cn;
        colnorm_row<SL, NN>(H, R, cb, cn);
        const dv2 xv = __builtin_nontemporal_load(x + k), bv = __builtin_nontemporal_load(b + k);
        const dv2 xnv = (NN && R.hasN) ? x[H.noff + k] : dv2{0.0, 0.0};
        double ri, rj;
        a_row<NN>(H, R, make_double2(xv.x, xv.y), make_double2(xnv.x, xnv.y), ri, rj);
        double2 gb, gn;
        at_row<NN>(H, R, ri - bv.x, rj - bv.y, gb, gn);
        const double vi = beta * cb.x, vj = beta * cb.y;
        dv2 xn;
        xn.x = soft_threshold<double>(xv.x - gb.x / vi, H.tau / vi);
        xn.y = soft_threshold<double>(xv.y - gb.y / vj, H.tau / vj);
        __builtin_nontemporal_store(pcdm_pick(H, k, step, thr, xn, xv), x + k);
        if (NN && R.hasN) {
            const double wi = beta * cn.x, wj = beta * cn.y;
            dv2 xnn;
            xnn.x = soft_threshold<double>(xnv.x - gn.x / wi, H.tau / wi);
            xnn.y = soft_threshold<double>(xnv.y - gn.y / wj, H.tau / wj);
            x[H.noff + k] = pcdm_pick(H, H.noff + k, step, thr, xnn, xnv);
        }
    }
}

// ---- CG-Newton ---------------------------------------------------------------
// M = (diag(A^T A) + d)^{-1}, the Jacobi preconditioner, on the pair
__device__ __forceinline__ dv2 precond(double2 cn, dv2 d) {
    dv2 m;
    m.x = 1.0 / (cn.x + d.x);
    m.y = 1.0 / (cn.y + d.y);
    return m;
}

// H p = A^T (A p) + d p on a row pair's coordinates (B's pair and, for IGen2
// rows, N~'s pair)
template <int NN>
__device__ __forceinline__ void hess_row(const SgtK& H, const Row& R, dv2 pb, dv2 pn, dv2 db, dv2 dn, dv2& hb,
                                         dv2& hn) {
    double yi, yj;
    a_row<NN>(H, R, make_double2(pb.x, pb.y), make_double2(pn.x, pn.y), yi, yj);
    double2 gb, gn;
    at_row<NN>(H, R, yi, yj, gb, gn);
    hb.x = gb.x + db.x * pb.x;
    hb.y = gb.y + db.y * pb.y;
    hn.x = gn.x + dn.x * pn.x;
    hn.y = gn.y + dn.y * pn.y;
}

// gradient of tau psi_mu at x plus a = A^T r, and the Hessian diagonal d
__device__ __forceinline__ void newton_terms(const SgtK& H, double mu, int primal, dv2 x, dv2 gd, double2 a,
                                             dv2& grad, dv2& d) {
    const double wi = sqrt(mu * mu + x.x * x.x), wj = sqrt(mu * mu + x.y * x.y);
    grad.x = H.tau * x.x / wi + a.x;
    grad.y = H.tau * x.y / wj + a.y;
    if (primal) {
        d.x = H.tau * mu * mu / (wi * wi * wi);
        d.y = H.tau * mu * mu / (wj * wj * wj);
    } else {
        d.x = H.tau * (1.0 - x.x * gd.x / wi) / wi;
        d.y = H.tau * (1.0 - x.y * gd.y / wj) / wj;
    }
}

// Start of a Newton step at x: grad f_mu = tau x / w + A^T (A x - b), the
// Hessian diagonal d (primal: tau mu^2 / w^3; primal-dual: tau (1 - x gd / w) / w),
// and PCG's start from dx = 0: r = -grad, u = M r.
// part = (r.u, u.Hu, r.r | max |grad|).
template <int SL, int NN>
__global__ __launch_bounds__(kHB) void kh_setup(SgtK H, const dv2* __restrict__ x, const dv2* __restrict__ gd,
                                                const double2* __restrict__ b, double mu, int primal,
                                                dv2* __restrict__ d, dv2* __restrict__ r, double* __restrict__ part) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const dv2 z2 = {0.0, 0.0};
    for (int64_t k = gtid(); k < H.np; k += gstride()) {
        const Row R = load_row<SL, NN>(H, k);
        const bool hn = NN && R.hasN;
        const int64_t kn = H.noff + k;
        const dv2 xb = x[k], xn = hn ? x[kn] : z2;
        const dv2 gb = primal ? z2 : gd[k], gn = (primal || !hn) ? z2 : gd[kn];
        const double2 bv = b[k];
        double yi, yj;
        a_row<NN>(H, R, make_double2(xb.x, xb.y), make_double2(xn.x, xn.y), yi, yj);
        double2 ab, an;
        at_row<NN>(H, R, yi - bv.x, yj - bv.y, ab, an);
        dv2 grb, db, grn = z2, dn = z2;
        newton_terms(H, mu, primal, xb, gb, ab, grb, db);
        if (hn) newton_terms(H, mu, primal, xn, gn, an, grn, dn);
        double2 cb, cn;
        colnorm_row<SL, NN>(H, R, cb, cn);
        const dv2 rb = -grb, rn = -grn;
        const dv2 ub = precond(cb, db) * rb;
        const dv2 un = hn ? precond(cn, dn) * rn : z2;
        dv2 wb, wn;
        hess_row<NN>(H, R, ub, un, db, dn, wb, wn);
        d[k] = db;
        r[k] = rb;
        v[0] += rb.x * ub.x + rb.y * ub.y;
        v[1] += wb.x * ub.x + wb.y * ub.y;
        v[2] += rb.x * rb.x + rb.y * rb.y;
        v[3] = fmax(v[3], fmax(fabs(grb.x), fabs(grb.y)));
        if (hn) {
            d[kn] = dn;
            r[kn] = rn;
            v[0] += rn.x * un.x + rn.y * un.y;
            v[1] += wn.x * un.x + wn.y * un.y;
            v[2] += rn.x * rn.x + rn.y * rn.y;
            v[3] = fmax(v[3], fmax(fabs(grn.x), fabs(grn.y)));
        }
    }
    store_partials<4, 3>(v, part);
}

// PCG scalars after kh_setup: gamma = r.u, ||rhs||, the stop test
// ||r|| > rtol ||rhs|| before the first iteration, alpha = gamma / u.Hu.
__global__ __launch_bounds__(1024) void kh_cg_init(const double* __restrict__ part, int nb, HCg* cs, double rtol,
                                                   int maxit) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
        v[0] += part[4 * q];
        v[1] += part[4 * q + 1];
        v[2] += part[4 * q + 2];
        v[3] = fmax(v[3], part[4 * q + 3]);
    }
    block_reduce_stats<4, 3>(v);
    if (threadIdx.x == 0) {
        const double rn = sqrt(v[2]);
        cs->gamma = v[0];
        cs->rr0 = v[2];
        cs->stop = rtol * rn;
        cs->gmax = v[3];
        cs->beta = 0.0;
        cs->iters = 0;
        cs->alpha = v[1] > 0.0 ? v[0] / v[1] : 0.0;
        cs->done = (maxit <= 0 || !(rn > cs->stop) || !(v[1] > 0.0)) ? 1 : 0;
    }
}

template <bool NT>
__device__ __forceinline__ dv2 ld2(const dv2* p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT>
__device__ __forceinline__ void st2(dv2 v, dv2* p) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// One PCG iteration: u = M r, p = u + beta p, dx += alpha p, r -= alpha H p,
// then for the next iteration u = M r, w = H u; part = (r.u, w.u, r.r).
// first: p and dx are not read (beta = 0, dx = 0).  U row pairs per thread
// per trip (B's loads issued together), NT: nontemporal accesses.
template <int SL, int NN, int U, bool NT>
__global__ __launch_bounds__(kHB) void kh_cg_iter(SgtK H, dv2* __restrict__ dx, dv2* __restrict__ r,
                                                  dv2* __restrict__ p, const dv2* __restrict__ d, int first,
                                                  const HCg* __restrict__ cs, double* __restrict__ part) {
    if (cs->done) return;
    const double a = cs->alpha, be = cs->beta;
    const dv2 z2 = {0.0, 0.0};
    double v[3] = {0.0, 0.0, 0.0};
    const int64_t np = H.np;
    const int64_t S = gstride();
    for (int64_t base = gtid(); base < np; base += U * S) {
        dv2 R[U], D[U], P[U], X[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t k = base + q * S;
            if (k < np) {
                R[q] = ld2<NT>(r + k);
                D[q] = ld2<NT>(d + k);
                if (!first) {
                    P[q] = ld2<NT>(p + k);
                    X[q] = ld2<NT>(dx + k);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int64_t k = base + q * S;
            if (k < np) {
                const Row Rw = load_row<SL, NN>(H, k);
                const bool hn = NN && Rw.hasN;
                const int64_t kn = H.noff + k;
                double2 cb, cn;
                colnorm_row<SL, NN>(H, Rw, cb, cn);
                dv2 Rn = z2, Dn = z2, Pn = z2, Xn = z2;
                if (hn) {
                    Rn = ld2<NT>(r + kn);
                    Dn = ld2<NT>(d + kn);
                    if (!first) {
                        Pn = ld2<NT>(p + kn);
                        Xn = ld2<NT>(dx + kn);
                    }
                }
                const dv2 mq = precond(cb, D[q]);
                const dv2 mqn = hn ? precond(cn, Dn) : z2;
                const dv2 u0 = mq * R[q], u0n = mqn * Rn;
                const dv2 pv = first ? u0 : u0 + be * P[q];
                const dv2 pvn = first ? u0n : u0n + be * Pn;
                dv2 sv, svn;
                hess_row<NN>(H, Rw, pv, pvn, D[q], Dn, sv, svn);
                const dv2 xo = first ? a * pv : X[q] + a * pv;
                const dv2 rn = R[q] - a * sv;
                const dv2 u1 = mq * rn;
                const dv2 xon = first ? a * pvn : Xn + a * pvn;
                const dv2 rnn = Rn - a * svn;
                const dv2 u1n = mqn * rnn;
                dv2 w1, w1n;
                hess_row<NN>(H, Rw, u1, u1n, D[q], Dn, w1, w1n);
                st2<NT>(pv, p + k);
                st2<NT>(xo, dx + k);
                st2<NT>(rn, r + k);
                v[0] += rn.x * u1.x + rn.y * u1.y;
                v[1] += w1.x * u1.x + w1.y * u1.y;
                v[2] += rn.x * rn.x + rn.y * rn.y;
                if (hn) {
                    st2<NT>(pvn, p + kn);
                    st2<NT>(xon, dx + kn);
                    st2<NT>(rnn, r + kn);
                    v[0] += rnn.x * u1n.x + rnn.y * u1n.y;
                    v[1] += w1n.x * u1n.x + w1n.y * u1n.y;
                    v[2] += rnn.x * rnn.x + rnn.y * rnn.y;
                }
            }
        }
    }
    store_partials<3, 3>(v, part);
}

// Textbook PCG (the oracle's recurrence), used where the single-reduction form
// loses accuracy: IGen2's N~ columns carry scales xi_j tau / |N_j^T e| over many
// orders of magnitude.  Update pass: dx += alpha p, r -= alpha H p, z = M r;
// part = (r.z, r.r).  first: p = M r (the start direction) is formed here and
// written, dx is not read.
template <int SL, int NN>
__global__ __launch_bounds__(kHB) void kh_tb_update(SgtK H, dv2* __restrict__ dx, dv2* __restrict__ r,
                                                    dv2* __restrict__ p, const dv2* __restrict__ d, int first,
                                                    const HCg* __restrict__ cs, double* __restrict__ part) {
    if (cs->done) return;
    const double a = cs->alpha;
    const dv2 z2 = {0.0, 0.0};
    double v[2] = {0.0, 0.0};
    for (int64_t k = gtid(); k < H.np; k += gstride()) {
        const Row Rw = load_row<SL, NN>(H, k);
        const bool hn = NN && Rw.hasN;
        const int64_t kn = H.noff + k;
        double2 cb, cn;
        colnorm_row<SL, NN>(H, Rw, cb, cn);
        const dv2 rb = r[k], db = d[k];
        const dv2 rn = hn ? r[kn] : z2, dn = hn ? d[kn] : z2;
        const dv2 mb = precond(cb, db), mn = hn ? precond(cn, dn) : z2;
        const dv2 pb = first ? mb * rb : p[k];
        const dv2 pn = hn ? (first ? mn * rn : p[kn]) : z2;
        dv2 hb, hnv;
        hess_row<NN>(H, Rw, pb, pn, db, dn, hb, hnv);
        const dv2 xb = first ? a * pb : dx[k] + a * pb;
        const dv2 r1 = rb - a * hb;
        const dv2 z1 = mb * r1;
        dx[k] = xb;
        r[k] = r1;
        if (first) p[k] = pb;
        v[0] += r1.x * z1.x + r1.y * z1.y;
        v[1] += r1.x * r1.x + r1.y * r1.y;
        if (hn) {
            const dv2 xn = first ? a * pn : dx[kn] + a * pn;
            const dv2 r1n = rn - a * hnv;
            const dv2 z1n = mn * r1n;
            dx[kn] = xn;
            r[kn] = r1n;
            if (first) p[kn] = pn;
            v[0] += r1n.x * z1n.x + r1n.y * z1n.y;
            v[1] += r1n.x * r1n.x + r1n.y * r1n.y;
        }
    }
    store_partials<2, 2>(v, part);
}

// beta = r.z / previous r.z; one iteration done; stop when ||r|| <= stop or at maxit
__global__ __launch_bounds__(1024) void kh_tb_beta(const double* __restrict__ part, int nb, HCg* cs, int maxit) {
    if (cs->done) return;
    double v[2] = {0.0, 0.0};
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
        v[0] += part[2 * q];
        v[1] += part[2 * q + 1];
    }
    block_reduce_stats<2, 2>(v);
    if (threadIdx.x == 0) {
        cs->iters += 1;
        if (cs->iters >= maxit || !(sqrt(v[1]) > cs->stop)) {
            cs->done = 1;
            return;
        }
        cs->beta = v[0] / cs->gamma;
        cs->gamma = v[0];
    }
}

// Direction pass: p = M r + beta p; part = p.Hp of the new p
template <int SL, int NN>
__global__ __launch_bounds__(kHB) void kh_tb_dir(SgtK H, const dv2* __restrict__ r, dv2* __restrict__ p,
                                                 const dv2* __restrict__ d, const HCg* __restrict__ cs,
                                                 double* __restrict__ part) {
    if (cs->done) return;
    const double be = cs->beta;
    const dv2 z2 = {0.0, 0.0};
    double v[1] = {0.0};
    for (int64_t k = gtid(); k < H.np; k += gstride()) {
        const Row Rw = load_row<SL, NN>(H, k);
        const bool hn = NN && Rw.hasN;
        const int64_t kn = H.noff + k;
        double2 cb, cn;
        colnorm_row<SL, NN>(H, Rw, cb, cn);
        const dv2 db = d[k], dn = hn ? d[kn] : z2;
        const dv2 pb = precond(cb, db) * r[k] + be * p[k];
        const dv2 pn = hn ? precond(cn, dn) * r[kn] + be * p[kn] : z2;
        dv2 hb, hnv;
        hess_row<NN>(H, Rw, pb, pn, db, dn, hb, hnv);
        p[k] = pb;
        v[0] += pb.x * hb.x + pb.y * hb.y;
        if (hn) {
            p[kn] = pn;
            v[0] += pn.x * hnv.x + pn.y * hnv.y;
        }
    }
    store_partials<1, 1>(v, part);
}

// alpha = r.z / p.Hp
__global__ __launch_bounds__(1024) void kh_tb_alpha(const double* __restrict__ part, int nb, HCg* cs) {
    if (cs->done) return;
    double v[1] = {0.0};
    for (int q = threadIdx.x; q < nb; q += blockDim.x) v[0] += part[q];
    block_reduce_stats<1, 1>(v);
    if (threadIdx.x == 0) {
        if (v[0] > 0.0)
            cs->alpha = cs->gamma / v[0];
        else
            cs->done = 1;  // no curvature left along p
    }
}

// One iteration done: stop when ||r|| <= stop or at maxit; else
// beta = gamma' / gamma, alpha = gamma' / (w.u - beta gamma' / alpha).
__global__ __launch_bounds__(1024) void kh_cg_next(const double* __restrict__ part, int nb, HCg* cs, int maxit) {
    if (cs->done) return;
    double v[3] = {0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
        v[0] += part[3 * q];
        v[1] += part[3 * q + 1];
        v[2] += part[3 * q + 2];
    }
    block_reduce_stats<3, 3>(v);
    if (threadIdx.x == 0) {
        cs->iters += 1;
        if (cs->iters >= maxit || !(sqrt(v[2]) > cs->stop)) {
            cs->done = 1;
            return;
        }
        const double be = v[0] / cs->gamma;
        const double den = v[1] - be * v[0] / cs->alpha;
        if (!(den > 0.0)) {  // no curvature left along the next direction
            cs->done = 1;
            return;
        }
        cs->beta = be;
        cs->alpha = v[0] / den;
        cs->gamma = v[0];
    }
}

// Line search terms at x along dx, for the step lengths a0 2^-t, t < kLsBatch:
// part = (sum psi(x), sum r(x)^2, grad . dx, sum psi(x + a_t dx) [t], sum r(x + a_t dx)^2 [t])
// with psi(v) = sqrt(mu^2 + v^2) - mu and r(v) = A v - b.
__device__ __forceinline__ double psi2(double mu, double a, double b) {
    return (sqrt(mu * mu + a * a) - mu) + (sqrt(mu * mu + b * b) - mu);
}

template <int SL, int NN>
__global__ __launch_bounds__(kHB) void kh_ls(SgtK H, const dv2* __restrict__ x, const dv2* __restrict__ dx,
                                             const double2* __restrict__ b, double mu, double a0,
                                             double* __restrict__ part) {
    double v[kLsStats];
#pragma unroll
    for (int q = 0; q < kLsStats; ++q) v[q] = 0.0;
    const dv2 z2 = {0.0, 0.0};
    for (int64_t k = gtid(); k < H.np; k += gstride()) {
        const Row R = load_row<SL, NN>(H, k);
        const bool hn = NN && R.hasN;
        const int64_t kn = H.noff + k;
        const dv2 xb = x[k], sb = dx[k];
        const dv2 xn = hn ? x[kn] : z2, sn = hn ? dx[kn] : z2;
        const double2 bv = b[k];
        double yi, yj;
        a_row<NN>(H, R, make_double2(xb.x, xb.y), make_double2(xn.x, xn.y), yi, yj);
        const double ri = yi - bv.x, rj = yj - bv.y;
        double2 ab, an;
        at_row<NN>(H, R, ri, rj, ab, an);
        const double wi = sqrt(mu * mu + xb.x * xb.x), wj = sqrt(mu * mu + xb.y * xb.y);
        v[0] += (wi - mu) + (wj - mu);
        v[1] += ri * ri + rj * rj;
        v[2] += (H.tau * xb.x / wi + ab.x) * sb.x + (H.tau * xb.y / wj + ab.y) * sb.y;
        if (hn) {
            const double wni = sqrt(mu * mu + xn.x * xn.x), wnj = sqrt(mu * mu + xn.y * xn.y);
            v[0] += (wni - mu) + (wnj - mu);
            v[2] += (H.tau * xn.x / wni + an.x) * sn.x + (H.tau * xn.y / wnj + an.y) * sn.y;
        }
        double a = a0;
#pragma unroll
        for (int t = 0; t < kLsBatch; ++t) {
            const dv2 ub = xb + a * sb, un = xn + a * sn;
            double qi, qj;
            a_row<NN>(H, R, make_double2(ub.x, ub.y), make_double2(un.x, un.y), qi, qj);
            qi -= bv.x;
            qj -= bv.y;
            v[3 + t] += psi2(mu, ub.x, ub.y);
            if (hn) v[3 + t] += psi2(mu, un.x, un.y);
            v[3 + kLsBatch + t] += qi * qi + qj * qj;
            a *= 0.5;
        }
    }
    store_partials<kLsStats, kLsStats>(v, part);
}

// dual update of the primal-dual diagonal at the old x (with the full
// direction), then x += a dx
__global__ __launch_bounds__(kHB) void kh_step(int64_t np, double2* __restrict__ x, double2* __restrict__ gd,
                                               const double2* __restrict__ dx, double a, double mu, int primal) {
    for (int64_t k = gtid(); k < np; k += gstride()) {
        const double2 xv = x[k], sv = dx[k];
        if (!primal) {
            const double2 g0 = gd[k];
            const double wi = sqrt(mu * mu + xv.x * xv.x), wj = sqrt(mu * mu + xv.y * xv.y);
            const double g1i = g0.x + (-g0.x + xv.x / wi + (1.0 - xv.x * g0.x / wi) * sv.x / wi);
            const double g1j = g0.y + (-g0.y + xv.y / wj + (1.0 - xv.y * g0.y / wj) * sv.y / wj);
            gd[k] = make_double2(fmin(1.0, fmax(-1.0, g1i)), fmin(1.0, fmax(-1.0, g1j)));
        }
        x[k] = make_double2(xv.x + a * sv.x, xv.y + a * sv.y);
    }
}

__global__ void kh_zero(double* __restrict__ v, int64_t n) {
    for (int64_t i = gtid(); i < n; i += gstride()) v[i] = 0.0;
}

int blocks_for(int64_t pairs) {
    int64_t g = (pairs + kHB - 1) / kHB;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, kHMaxBlocks));
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
bool is_fin(double v) { return std::isfinite(v); }

// Run f(std::integral_constant<int, SL>) for the instance's sigma law.
template <typename F>
void by_law(int law, F&& f) {
    if (law == L1LS_SIGMA_UNIFORM)
        f(std::integral_constant<int, 1>{});
    else
        f(std::integral_constant<int, 0>{});
}

// Run f(SL, NN) as integral constants: the sigma law and whether the
// instance is IGen2's (row pairs with N~ blocks).
template <typename F>
void by_kind(const SgtK& K, F&& f) {
    by_law(K.sigma_law, [&](auto c) {
        if (K.nnp > 0)
            f(c, std::integral_constant<int, 1>{});
        else
            f(c, std::integral_constant<int, 0>{});
    });
}

}  // namespace

struct l1ls_sgt {
    l1ls_sgt_params prm;
    SgtK k;
    double L = 0, fstar = 0, sigma_min = 0, sigma_max = 0;
    int device = 0;
    double* b = nullptr;  // n: the top n entries of b (rows n..m-1 of b are zero)
    double* part = nullptr;
    unsigned long long* hist = nullptr;  // radix-select histogram
    DevArena arena;
    // HIP-event times of the last solve with opts.time_kernels set:
    // [0] PCG iteration pass (CG-Newton) or iteration pass (FISTA),
    // [1] line-search pass (CG-Newton) or gap pass (FISTA), [2] Newton setup pass
    mutable double kt_ms[3] = {0, 0, 0};
    mutable int64_t kt_calls[3] = {0, 0, 0};
    ~l1ls_sgt() { arena.release(); }
};

namespace {

// Sum of NS statistics over nb partial slots in fixed order (the last
// NS - nsum of them take the maximum).
l1ls_status host_stats(const double* part, int ns, int nsum, int nb, hipStream_t s, double* out) {
    std::vector<double> h((size_t)ns * nb);
    HIP_TRY(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int q = 0; q < ns; ++q) out[q] = q < nsum ? 0.0 : -INFINITY;
    for (int bk = 0; bk < nb; ++bk)
        for (int q = 0; q < ns; ++q) {
            const double v = h[(size_t)ns * bk + q];
            out[q] = q < nsum ? out[q] + v : std::max(out[q], v);
        }
    return L1LS_OK;
}

l1ls_status sgt_gap(const l1ls_sgt* H, double tau, const double* x, hipStream_t s, double* P, double* D,
                    double* gap, double* part) {
    const int nb = blocks_for(H->k.n / 2);
    SgtK K = H->k;
    by_kind(K, [&](auto c, auto nn) {
        hipLaunchKernelGGL((kh_gap<decltype(c)::value, decltype(nn)::value>), dim3(nb), dim3(kHB), 0, s, K,
                           (const double2*)x,
                           (const double2*)H->b, part);
    });
    HIP_TRY(hipGetLastError());
    double t[4];
    L1LS_TRY(host_stats(part, 4, 3, nb, s, t));
    *P = tau * t[0] + 0.5 * t[1];
    const double theta = (t[3] <= tau) ? 1.0 : tau / t[3];
    *D = -0.5 * theta * theta * t[1] - theta * t[2];
    *gap = (*P - *D) / std::fabs(*P);
    if (!is_fin(*P) || !is_fin(*D)) return L1LS_E_NONFINITE;
    return L1LS_OK;
}

l1ls_status sgt_err(const l1ls_sgt* H, const double* x, hipStream_t s, double* out, double* part) {
    const int nb = blocks_for(H->k.n / 2);
    by_kind(H->k, [&](auto c, auto nn) {
        hipLaunchKernelGGL((kh_err<decltype(c)::value, decltype(nn)::value>), dim3(nb), dim3(kHB), 0, s, H->k,
                           (const double2*)x, part);
    });
    HIP_TRY(hipGetLastError());
    double t[2];
    L1LS_TRY(host_stats(part, 2, 2, nb, s, t));
    *out = (t[1] > 0) ? std::sqrt(t[0] / t[1]) : std::sqrt(t[0]);
    return L1LS_OK;
}

// The element of rank `rank` (1-based) in the order (|x_i|, i) of OsGen3's
// unselected x: 8 passes over the magnitude bits, then 4 over the index bits
// of the elements with that magnitude.
l1ls_status osgen3_select(l1ls_sgt* H, int64_t rank, hipStream_t s, uint64_t* bits_out, int64_t* idx_out) {
    const int nb = blocks_for(H->k.n / 2);
    unsigned long long h[kSelBins];
    auto pass = [&](int by_index, uint64_t value, uint64_t prefix, uint64_t mask, int shift) -> l1ls_status {
        HIP_TRY(hipMemsetAsync(H->hist, 0, sizeof(h), s));
        by_law(H->k.sigma_law, [&](auto c) {
            hipLaunchKernelGGL(kh_select_hist<decltype(c)::value>, dim3(nb), dim3(kHB), 0, s, H->k, by_index,
                               value, prefix, mask, shift, H->hist);
        });
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(h, H->hist, sizeof(h), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return L1LS_OK;
    };
    // rank within the current bucket, walked digit by digit from the top
    auto descend = [&](uint64_t& prefix, uint64_t& mask, int shift, int64_t& left) -> l1ls_status {
        int d = 0;
        for (; d < kSelBins; ++d) {
            if (left <= (int64_t)h[d]) break;
            left -= (int64_t)h[d];
        }
        if (d == kSelBins) return L1LS_E_STATE;  // counts disagree with the rank
        prefix |= (uint64_t)d << shift;
        mask |= (uint64_t)0xff << shift;
        return L1LS_OK;
    };
    int64_t left = rank;
    uint64_t prefix = 0, mask = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        L1LS_TRY(pass(0, 0, prefix, mask, shift));
        L1LS_TRY(descend(prefix, mask, shift, left));
    }
    const uint64_t value = prefix;
    uint64_t ip = 0, im = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
        L1LS_TRY(pass(1, value, ip, im, shift));
        L1LS_TRY(descend(ip, im, shift, left));
    }
    *bits_out = value;
    *idx_out = (int64_t)ip;
    return L1LS_OK;
}

bool valid_params(const l1ls_sgt_params* p) {
    const int64_t n = p->n, m = p->m;
    if (n < 2 || n % 2 || n > kSgtMaxN || m < 2 || m % 2 || p->s < 0 || p->s > std::min(m, n)) return false;
    // IGen2 (m < n): N~ has n - m <= m columns, x* lies in the first m, OsGen3 is for m >= n
    if (m < n && (n - m > m || p->xstar_law == L1LS_XSTAR_OSGEN3)) return false;
    if (!(p->tau > 0) || !is_fin(p->tau) || !is_fin(p->theta)) return false;
    if (p->sigma_law == L1LS_SIGMA_ALTERNATING) {
        if (!(p->sigma_odd > 0) || !(p->sigma_even > 0) || !is_fin(p->sigma_odd) || !is_fin(p->sigma_even))
            return false;
    } else if (p->sigma_law == L1LS_SIGMA_UNIFORM) {
        if (!(p->sigma_scale >= 0) || !(p->sigma_shift > 0) || !is_fin(p->sigma_scale) || !is_fin(p->sigma_shift))
            return false;
    } else {
        return false;
    }
    if (p->xstar_law == L1LS_XSTAR_TABLE1) {
        if (!is_fin(p->x_neg) || !is_fin(p->x_pos)) return false;
    } else if (p->xstar_law == L1LS_XSTAR_OSGEN) {
        if (!(p->gamma > 0) || !is_fin(p->gamma)) return false;
    } else if (p->xstar_law == L1LS_XSTAR_OSGEN3) {
        if (!(p->gamma > 0) || !is_fin(p->gamma) || p->s1 < 0 || p->s2 < 0 || p->s1 + p->s2 != p->s) return false;
    } else {
        return false;
    }
    return true;
}

}  // namespace

extern "C" void l1ls_sgt_params_default(int64_t n, uint64_t seed, l1ls_sgt_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->n = n;
    p->m = 2 * n;
    p->s = n / 1024;
    p->theta = 2.0 * M_PI / 3.0;
    p->sigma_odd = 0.1;
    p->sigma_even = 100.0;
    p->x_neg = -1.0e4;
    p->x_pos = 0.1;
    p->tau = 1.0;
    p->seed = seed;
    p->sigma_law = L1LS_SIGMA_ALTERNATING;
    p->sigma_scale = 1.0;
    p->sigma_shift = 0.1;
    p->xstar_law = L1LS_XSTAR_TABLE1;
    p->gamma = 1.0;
    p->s1 = p->s / 2;
    p->s2 = p->s - p->s1;
}

extern "C" size_t l1ls_sgt_bytes(int64_t n) {
    if (n < 2) return 0;
    return (size_t)n * sizeof(double) + (size_t)kHMaxBlocks * kLsStats * sizeof(double) + 8192;
}

extern "C" size_t l1ls_sgt_solve_bytes(int64_t n) {
    if (n < 2) return 0;
    return 5 * (size_t)n * sizeof(double) + (size_t)kHMaxBlocks * kLsStats * sizeof(double) + 4096;
}

extern "C" l1ls_status l1ls_sgt_generate(const l1ls_sgt_params* p, void* stream, l1ls_sgt** out) {
    if (!p || !out) return L1LS_E_ARG;
    *out = nullptr;
    if (!valid_params(p)) return L1LS_E_ARG;
    const int64_t n = p->n;
    hipStream_t s = (hipStream_t)stream;
    auto* H = new (std::nothrow) l1ls_sgt();
    if (!H) return L1LS_E_NOMEM;
    H->prm = *p;
    SgtK& K = H->k;
    std::memset(&K, 0, sizeof(K));
    K.n = n;
    K.s = p->s;
    K.s1 = p->s1;
    K.s2 = p->s2;
    K.np = std::min(p->m, n) / 2;
    K.nnp = n > p->m ? (n - p->m) / 2 : 0;
    K.noff = p->m / 2;
    K.nsup = std::min(p->m, n);
    K.sigma_law = p->sigma_law;
    K.xstar_law = p->xstar_law;
    K.c = std::cos(p->theta);
    K.sn = std::sin(p->theta);
    K.so = p->sigma_odd;
    K.se = p->sigma_even;
    K.cn0 = K.so * K.so * K.c * K.c + K.se * K.se * K.sn * K.sn;
    K.cn1 = K.so * K.so * K.sn * K.sn + K.se * K.se * K.c * K.c;
    K.scale = p->sigma_scale;
    K.shift = p->sigma_shift;
    K.tau = p->tau;
    K.xneg = p->x_neg;
    K.xpos = p->x_pos;
    K.gamma = p->gamma;
    K.key = seed_key(p->seed);
    auto fail = [&](l1ls_status st) {
        (void)hipStreamSynchronize(s);
        delete H;
        return st;
    };
    if (hipGetDevice(&H->device) != hipSuccess) return fail(L1LS_E_HIP);
    l1ls_status st = H->arena.alloc(&H->b, (size_t)n);
    if (st == L1LS_OK) st = H->arena.alloc(&H->part, (size_t)kHMaxBlocks * kLsStats);
    if (st == L1LS_OK) st = H->arena.alloc(&H->hist, (size_t)kSelBins);
    double* csw = nullptr;
    if (st == L1LS_OK && K.nnp > 0) st = H->arena.alloc(&csw, (size_t)(2 * K.nnp));
    if (st != L1LS_OK) return fail(st);
    K.cs = csw;
    if (K.xstar_law == L1LS_XSTAR_OSGEN3) {
        // the s1 smallest: up to rank s1; the s2 largest: from rank n - s2 + 1
        if (K.s1 > 0) {
            st = osgen3_select(H, K.s1, s, &K.t1_bits, &K.t1_idx);
            K.has1 = 1;
        }
        if (st == L1LS_OK && K.s2 > 0) {
            st = osgen3_select(H, n - K.s2 + 1, s, &K.t2_bits, &K.t2_idx);
            K.has2 = 1;
        }
        if (st != L1LS_OK) return fail(st);
    }
    const int nb = blocks_for(n / 2);
    by_kind(K, [&](auto c, auto nn) {
        hipLaunchKernelGGL((kh_generate<decltype(c)::value, decltype(nn)::value>), dim3(nb), dim3(kHB), 0, s, K,
                           (double2*)H->b, (double2*)csw, H->part);
    });
    if (hipGetLastError() != hipSuccess) return fail(L1LS_E_HIP);
    double t[5] = {0, 0, 0, 0, 0};
    st = host_stats(H->part, 5, 2, nb, s, t);
    if (st != L1LS_OK) return fail(st);
    H->sigma_max = t[2];
    H->sigma_min = -t[3];
    H->L = t[4];  // lambda_max(A A^T): sigma_max^2, or the largest 2 x 2 row block of IGen2's [B, N~]
    // f* = tau ||x*||_1 + 0.5 ||e||^2; Table 1's ||x*||_1 in closed form
    double l1 = t[1];
    if (K.xstar_law == L1LS_XSTAR_TABLE1) {
        const int64_t nneg = p->s / 2, npos = p->s - nneg;
        l1 = (double)nneg * std::fabs(p->x_neg) + (double)npos * std::fabs(p->x_pos);
    }
    H->fstar = p->tau * l1 + 0.5 * t[0];
    *out = H;
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_sgt_describe(const l1ls_sgt* H, l1ls_sgt_desc* out) {
    if (!H || !out) return L1LS_E_ARG;
    std::memset(out, 0, sizeof(*out));
    out->params = H->prm;
    out->L = H->L;
    out->f_star = H->fstar;
    out->c = H->k.c;
    out->s_rot = H->k.sn;
    out->b_dev = H->b;
    out->sigma_min = H->sigma_min;
    out->sigma_max = H->sigma_max;
    out->colscale_dev = H->k.cs;
    return L1LS_OK;
}

extern "C" void l1ls_sgt_free(l1ls_sgt* H) {
    if (!H) return;
    int cur = 0;
    const bool sw = hipGetDevice(&cur) == hipSuccess && cur != H->device;
    if (sw) (void)hipSetDevice(H->device);
    (void)hipDeviceSynchronize();
    delete H;
    if (sw) (void)hipSetDevice(cur);
}

extern "C" l1ls_status l1ls_sgt_planted(const l1ls_sgt* H, double* x_star_dev, double* g_dev, void* stream) {
    if (!H || (!x_star_dev && !g_dev)) return L1LS_E_ARG;
    by_kind(H->k, [&](auto c, auto nn) {
        hipLaunchKernelGGL((kh_planted<decltype(c)::value, decltype(nn)::value>), dim3(blocks_for(H->k.n / 2)),
                           dim3(kHB), 0,
                           (hipStream_t)stream, H->k, x_star_dev, g_dev);
    });
    HIP_TRY(hipGetLastError());
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_sgt_apply(const l1ls_sgt* H, int32_t trans, const double* in_dev, double* out_dev,
                                      void* stream) {
    if (!H || !in_dev || !out_dev || (trans != 0 && trans != 1)) return L1LS_E_ARG;
    if (!aligned16(in_dev) || !aligned16(out_dev)) return L1LS_E_ARG;
    const int64_t m = H->prm.m;
    const int nb = blocks_for(trans ? H->k.n / 2 : m / 2);
    by_kind(H->k, [&](auto c, auto nn) {
        hipLaunchKernelGGL((kh_apply<decltype(c)::value, decltype(nn)::value>), dim3(nb), dim3(kHB), 0,
                           (hipStream_t)stream, H->k, m,
                           (int)trans, (const double2*)in_dev, (double2*)out_dev);
    });
    HIP_TRY(hipGetLastError());
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_sgt_objective_gap(const l1ls_sgt* H, double tau, const double* x_dev, double* P,
                                              double* D, double* gap, void* stream) {
    if (!H || !x_dev || !P || !D || !gap || !(tau > 0) || !is_fin(tau)) return L1LS_E_ARG;
    if (!aligned16(x_dev)) return L1LS_E_ARG;
    return sgt_gap(H, tau, x_dev, (hipStream_t)stream, P, D, gap, H->part);
}

extern "C" l1ls_status l1ls_sgt_kappa_rho(const l1ls_sgt* H, double rho, double* kappa, void* stream) {
    if (!H || !kappa || !(rho >= 0) || !is_fin(rho)) return L1LS_E_ARG;
    if (H->k.nnp > 0) return L1LS_E_UNSUPPORTED;  // A^T A is singular for m < n (section 5)
    hipStream_t s = (hipStream_t)stream;
    const int nb = blocks_for(H->k.n / 2);
    by_law(H->k.sigma_law, [&](auto c) {
        hipLaunchKernelGGL(kh_kappa<decltype(c)::value>, dim3(nb), dim3(kHB), 0, s, H->k, rho, H->part);
    });
    HIP_TRY(hipGetLastError());
    double t[2];
    L1LS_TRY(host_stats(H->part, 2, 2, nb, s, t));
    *kappa = (t[1] > 0) ? std::sqrt(t[0] / t[1]) : INFINITY;
    return L1LS_OK;
}

namespace {

// t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2, without contraction
double next_t_sgt(double t) {
#pragma clang fp contract(off)
    return (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
}

}  // namespace

extern "C" l1ls_status l1ls_sgt_solve_fista(const l1ls_sgt* H, const l1ls_solve_opts* o, double* x,
                                            l1ls_report* rep) {
    if (!H || !o || !x) return L1LS_E_ARG;
    if (o->max_iter < 0 || !aligned16(x) || (o->x0_dev && !aligned16(o->x0_dev))) return L1LS_E_ARG;
    if (o->precision != L1LS_F64 || o->polish != 0) return L1LS_E_UNSUPPORTED;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)o->stream;
    const double tau = o->tau > 0 ? o->tau : H->prm.tau;
    const double L = o->L > 0 ? o->L : H->L;
    const int check = std::max(1, o->check_every);
    if (!is_fin(tau) || !is_fin(L) || !(L > 0)) return L1LS_E_ARG;
    SgtK K = H->k;
    K.tau = tau;
    const int64_t n = K.n;
    const int nb = blocks_for(n / 2);
    const bool tk = o->time_kernels != 0;
    DevArena W;
    double *xb = nullptr, *part = nullptr;
    std::vector<hipEvent_t> ev;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        W.release();
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    };
    auto run = [&]() -> l1ls_status {
        L1LS_TRY(W.alloc(&xb, (size_t)n));
        L1LS_TRY(W.alloc(&part, (size_t)kHMaxBlocks * 4));
        if (tk) {
            for (int q = 0; q < 3; ++q) {
                H->kt_ms[q] = 0;
                H->kt_calls[q] = 0;
            }
            ev.resize(2 * (size_t)check + 2);
            for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
        }
        auto elapsed = [&](int a, int b) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
            return (double)ms;
        };
        if (o->x0_dev) {
            if (o->x0_dev != x) HIP_TRY(hipMemcpyAsync(x, o->x0_dev, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        } else {
            hipLaunchKernelGGL(kh_zero, dim3(nb), dim3(kHB), 0, s, x, n);
        }
        // x_{-1} = x_0: the first step's momentum term is 0 (beta_0 = 0)
        HIP_TRY(hipMemcpyAsync(xb, x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        double* cur = x;   // x_{k-1}
        double* old = xb;  // x_{k-2}, receives x_k
        double t = 1.0, beta = 0.0, P = 0, D = 0, gap = INFINITY;
        int64_t k = 0;
        bool stop = false;
        while (k < o->max_iter && !stop) {
            const int64_t batch = std::min<int64_t>(check - (k % check), o->max_iter - k);
            for (int64_t q = 0; q < batch; ++q) {
                if (tk) HIP_TRY(hipEventRecord(ev[2 * q], s));
                by_kind(K, [&](auto c, auto nn) {
                    hipLaunchKernelGGL((kh_fista<decltype(c)::value, decltype(nn)::value>), dim3(nb), dim3(kHB), 0,
                                       s, K, (const dv2*)cur,
                                       (dv2*)old, (const dv2*)H->b, beta, L, tau / L);
                });
                if (tk) HIP_TRY(hipEventRecord(ev[2 * q + 1], s));
                const double t_next = next_t_sgt(t);
                beta = (t - 1.0) / t_next;
                t = t_next;
                std::swap(cur, old);
                ++k;
            }
            HIP_TRY(hipGetLastError());
            if (tk) HIP_TRY(hipEventRecord(ev[2 * check], s));
            L1LS_TRY(sgt_gap(H, tau, cur, s, &P, &D, &gap, part));
            if (tk) {
                HIP_TRY(hipEventRecord(ev[2 * check + 1], s));
                HIP_TRY(hipEventSynchronize(ev[2 * check + 1]));
                for (int64_t q = 0; q < batch; ++q) H->kt_ms[0] += elapsed((int)(2 * q), (int)(2 * q + 1));
                H->kt_calls[0] += batch;
                H->kt_ms[1] += elapsed(2 * check, 2 * check + 1);
                H->kt_calls[1] += 1;
            }
            if ((o->rel_gap_tol > 0 && gap <= o->rel_gap_tol) || (o->f_target > 0 && P <= o->f_target)) stop = true;
        }
        if (cur != x) HIP_TRY(hipMemcpyAsync(x, cur, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        if (k == 0) L1LS_TRY(sgt_gap(H, tau, x, s, &P, &D, &gap, part));
        l1ls_report rr;
        std::memset(&rr, 0, sizeof(rr));
        rr.iterations = k;
        rr.primal = P;
        rr.dual = D;
        rr.rel_gap = gap;
        L1LS_TRY(sgt_err(H, x, s, &rr.rel_err, part));
        rr.converged = stop ? 1 : 0;
        rr.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (rep) *rep = rr;
        return stop ? L1LS_OK : L1LS_NOT_CONVERGED;
    };
    const l1ls_status st = run();
    cleanup();
    return st;
}

extern "C" l1ls_status l1ls_sgt_solve_pcdm(const l1ls_sgt* H, const l1ls_solve_opts* o, double* x,
                                           l1ls_report* rep) {
    if (!H || !o || !x) return L1LS_E_ARG;
    if (o->max_iter < 0 || !aligned16(x) || (o->x0_dev && !aligned16(o->x0_dev))) return L1LS_E_ARG;
    if (o->precision != L1LS_F64 || o->polish != 0) return L1LS_E_UNSUPPORTED;
    if (!(o->max_iter < ((int64_t)1 << 32))) return L1LS_E_ARG;  // the step is a Philox counter word
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)o->stream;
    const double tau = o->tau > 0 ? o->tau : H->prm.tau;
    const double p = (o->pcdm_p > 0 && o->pcdm_p < 1) ? o->pcdm_p : 1.0;
    const int check = std::max(1, o->check_every);
    if (!is_fin(tau)) return L1LS_E_ARG;
    // omega nonzeros per row (2, or 4 in IGen2's rows with an N~ block); beta of a
    // doubly uniform sampling with E|S| = n p
    const int omega = H->k.nnp > 0 ? 4 : 2;
    const double beta = 1.0 + (omega - 1) * p;
    const uint64_t thr = p >= 1.0 ? ((uint64_t)1 << 32) : (uint64_t)(p * 4294967296.0);
    SgtK K = H->k;
    K.tau = tau;
    const int64_t n = K.n;
    const int nb = blocks_for(n / 2);
    const bool tk = o->time_kernels != 0;
    DevArena W;
    double* part = nullptr;
    std::vector<hipEvent_t> ev;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(s);
        W.release();
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    };
    auto run = [&]() -> l1ls_status {
        L1LS_TRY(W.alloc(&part, (size_t)kHMaxBlocks * 4));
        if (tk) {
            for (int q = 0; q < 3; ++q) {
                H->kt_ms[q] = 0;
                H->kt_calls[q] = 0;
            }
            ev.resize(2 * (size_t)check);
            for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
        }
        if (o->x0_dev) {
            if (o->x0_dev != x) HIP_TRY(hipMemcpyAsync(x, o->x0_dev, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        } else {
            hipLaunchKernelGGL(kh_zero, dim3(nb), dim3(kHB), 0, s, x, n);
        }
        double P = 0, D = 0, gap = INFINITY;
        int64_t k = 0;
        bool stop = false;
        while (k < o->max_iter && !stop) {
            const int64_t batch = std::min<int64_t>(check - (k % check), o->max_iter - k);
            for (int64_t q = 0; q < batch; ++q) {
                if (tk) HIP_TRY(hipEventRecord(ev[2 * q], s));
                by_kind(K, [&](auto c, auto nn) {
                    hipLaunchKernelGGL((kh_pcdm<decltype(c)::value, decltype(nn)::value>), dim3(nb), dim3(kHB), 0,
                                       s, K, (dv2*)x,
                                       (const dv2*)H->b, beta, thr, (uint32_t)k);
                });
                if (tk) HIP_TRY(hipEventRecord(ev[2 * q + 1], s));
                ++k;
            }
            HIP_TRY(hipGetLastError());
            L1LS_TRY(sgt_gap(H, tau, x, s, &P, &D, &gap, part));
            if (tk) {
                for (int64_t q = 0; q < batch; ++q) {
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, ev[2 * q], ev[2 * q + 1]);
                    H->kt_ms[0] += ms;
                }
                H->kt_calls[0] += batch;
            }
            if ((o->rel_gap_tol > 0 && gap <= o->rel_gap_tol) || (o->f_target > 0 && P <= o->f_target)) stop = true;
        }
        if (k == 0) L1LS_TRY(sgt_gap(H, tau, x, s, &P, &D, &gap, part));
        l1ls_report rr;
        std::memset(&rr, 0, sizeof(rr));
        rr.iterations = k;
        rr.primal = P;
        rr.dual = D;
        rr.rel_gap = gap;
        L1LS_TRY(sgt_err(H, x, s, &rr.rel_err, part));
        rr.converged = stop ? 1 : 0;
        rr.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (rep) *rep = rr;
        return stop ? L1LS_OK : L1LS_NOT_CONVERGED;
    };
    const l1ls_status st = run();
    cleanup();
    return st;
}

// CG-Newton state between l1ls_sgt_newton_step calls: the iterate x (the
// caller's buffer), the primal-dual variable gd and the PCG vectors.
struct l1ls_sgt_newton {
    static constexpr int kBatch = 8;  // PCG iterations enqueued between host checks
    static constexpr int kEv = 2 * kBatch + 2;
    const l1ls_sgt* H = nullptr;
    hipStream_t s = nullptr;
    SgtK K{};
    double tau = 1, mu = 1e-5, prtol = 0.1, gtol = 1e-9;
    int maxbt = 50, pcgmax = 1000, primal = 0, nb = 1;
    bool tk = false;
    double* x = nullptr;
    double *gd = nullptr, *dx = nullptr, *r = nullptr, *p = nullptr, *d = nullptr, *part = nullptr;
    HCg* cs = nullptr;
    DevArena W;
    hipEvent_t ev[kEv];
    int nev = 0;
    int64_t newton = 0, pcg_total = 0;
    double gnorm = INFINITY;
    bool converged = false;
    std::chrono::steady_clock::time_point t0;

    ~l1ls_sgt_newton() {
        (void)hipStreamSynchronize(s);  // nothing queued may still use the buffers
        W.release();
        for (int q = 0; q < nev; ++q) (void)hipEventDestroy(ev[q]);
    }
    double elapsed(int a, int b) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
        return (double)ms;
    }

    l1ls_status init(const l1ls_sgt* inst, const l1ls_solve_opts* o, double* xdev) {
        H = inst;
        x = xdev;
        s = (hipStream_t)o->stream;
        tau = o->tau > 0 ? o->tau : H->prm.tau;
        mu = o->mu > 0 ? o->mu : 1e-5;
        prtol = o->pcg_rtol > 0 ? o->pcg_rtol : 0.1;
        maxbt = o->max_backtrack > 0 ? o->max_backtrack : 50;
        pcgmax = o->pcg_maxit > 0 ? o->pcg_maxit : 1000;
        primal = o->hessian == 1 ? 1 : 0;
        gtol = (o->rel_gap_tol > 0 ? o->rel_gap_tol : 1e-9) * tau;
        tk = o->time_kernels != 0;
        if (!is_fin(tau) || !is_fin(mu)) return L1LS_E_ARG;
        K = H->k;
        K.tau = tau;
        const int64_t n = K.n;
        nb = blocks_for(n / 2);
        for (double** v : {&gd, &dx, &r, &p, &d}) L1LS_TRY(W.alloc(v, (size_t)n));
        L1LS_TRY(W.alloc(&part, (size_t)kHMaxBlocks * kLsStats));
        L1LS_TRY(W.alloc(&cs, 1));
        if (tk) {
            for (int q = 0; q < 3; ++q) {
                H->kt_ms[q] = 0;
                H->kt_calls[q] = 0;
            }
            for (; nev < kEv; ++nev) HIP_TRY(hipEventCreate(&ev[nev]));
        }
        t0 = std::chrono::steady_clock::now();
        if (o->x0_dev) {
            if (o->x0_dev != x) HIP_TRY(hipMemcpyAsync(x, o->x0_dev, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        } else {
            hipLaunchKernelGGL(kh_zero, dim3(nb), dim3(kHB), 0, s, x, n);
        }
        hipLaunchKernelGGL(kh_zero, dim3(nb), dim3(kHB), 0, s, gd, n);
        HIP_TRY(hipGetLastError());
        return L1LS_OK;
    }

    // PCG on the Newton system from dx = 0 (kh_setup has formed its start)
    l1ls_status pcg(HCg& c) {
        const int64_t n = K.n;
        if (c.done) hipLaunchKernelGGL(kh_zero, dim3(nb), dim3(kHB), 0, s, dx, n);  // no iteration writes dx
        int first = 1;
        while (!c.done) {
            const int before = c.iters;
            const int skip = first;  // the first iteration reads no p, dx: not timed
            for (int q = 0; q < kBatch; ++q) {
                if (tk) HIP_TRY(hipEventRecord(ev[2 * q], s));
                if (K.nnp > 0) {
                    // IGen2: the textbook recurrence (two passes per iteration)
                    by_law(K.sigma_law, [&](auto c) {
                        hipLaunchKernelGGL((kh_tb_update<decltype(c)::value, 1>), dim3(nb), dim3(kHB), 0, s, K,
                                           (dv2*)dx, (dv2*)r, (dv2*)p, (const dv2*)d, first, (const HCg*)cs, part);
                        hipLaunchKernelGGL(kh_tb_beta, dim3(1), dim3(1024), 0, s, part, nb, cs, pcgmax);
                        hipLaunchKernelGGL((kh_tb_dir<decltype(c)::value, 1>), dim3(nb), dim3(kHB), 0, s, K,
                                           (const dv2*)r, (dv2*)p, (const dv2*)d, (const HCg*)cs, part);
                        hipLaunchKernelGGL(kh_tb_alpha, dim3(1), dim3(1024), 0, s, part, nb, cs);
                    });
                    if (tk) HIP_TRY(hipEventRecord(ev[2 * q + 1], s));
                    first = 0;
                    continue;
                }
                by_kind(K, [&](auto c, auto nn) {
                    constexpr int NN = decltype(nn)::value;
                    hipLaunchKernelGGL((kh_cg_iter<decltype(c)::value, NN, NN ? 1 : kHU, kHNT>), dim3(nb),
                                       dim3(kHB), 0, s, K,
                                       (dv2*)dx, (dv2*)r, (dv2*)p, (const dv2*)d, first, (const HCg*)cs, part);
                });
                if (tk) HIP_TRY(hipEventRecord(ev[2 * q + 1], s));
                hipLaunchKernelGGL(kh_cg_next, dim3(1), dim3(1024), 0, s, part, nb, cs, pcgmax);
                first = 0;
            }
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipMemcpyAsync(&c, cs, sizeof(c), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (tk) {  // the passes that ran: one per iteration of this batch
                const int ran = c.iters - before;
                for (int q = skip; q < ran; ++q) H->kt_ms[0] += elapsed(2 * q, 2 * q + 1);
                H->kt_calls[0] += std::max(ran - skip, 0);
            }
        }
        pcg_total += c.iters;
        return L1LS_OK;
    }

    // Armijo backtracking on f_mu(x + a dx), a = 2^-t, kLsBatch lengths per pass;
    // a = 2^-maxbt when none of the maxbt lengths passes
    l1ls_status line_search(double* a_out) {
        const double armijo = 1e-4;
        double a = std::ldexp(1.0, -maxbt);
        bool found = false;
        for (int t0b = 0; t0b < maxbt && !found; t0b += kLsBatch) {
            const double a0 = std::ldexp(1.0, -t0b);
            if (tk) HIP_TRY(hipEventRecord(ev[2 * kBatch], s));
            by_kind(K, [&](auto c, auto nn) {
                hipLaunchKernelGGL((kh_ls<decltype(c)::value, decltype(nn)::value>), dim3(nb), dim3(kHB), 0, s, K,
                                   (const dv2*)x, (const dv2*)dx, (const double2*)H->b, mu, a0, part);
            });
            if (tk) HIP_TRY(hipEventRecord(ev[2 * kBatch + 1], s));
            HIP_TRY(hipGetLastError());
            double t[kLsStats];
            L1LS_TRY(host_stats(part, kLsStats, kLsStats, nb, s, t));
            if (tk) {
                H->kt_ms[1] += elapsed(2 * kBatch, 2 * kBatch + 1);
                H->kt_calls[1] += 1;
            }
            const double f0 = tau * t[0] + 0.5 * t[1];
            const double slope = t[2];
            for (int q = 0; q < kLsBatch && t0b + q < maxbt; ++q) {
                const double at = std::ldexp(1.0, -(t0b + q));
                const double ft = tau * t[3 + q] + 0.5 * t[3 + kLsBatch + q];
                if (ft <= f0 + armijo * at * slope) {
                    a = at;
                    found = true;
                    break;
                }
            }
        }
        *a_out = a;
        return L1LS_OK;
    }

    // up to k Newton steps; stops at ||grad f_mu||_inf <= gtol
    l1ls_status steps(int64_t k) {
        for (int64_t q = 0; q < k && !converged; ++q) {
            if (tk) HIP_TRY(hipEventRecord(ev[2 * kBatch], s));
            by_kind(K, [&](auto c, auto nn) {
                hipLaunchKernelGGL((kh_setup<decltype(c)::value, decltype(nn)::value>), dim3(nb), dim3(kHB), 0, s,
                                   K, (const dv2*)x, (const dv2*)gd, (const double2*)H->b, mu, primal, (dv2*)d,
                                   (dv2*)r, part);
            });
            if (tk) HIP_TRY(hipEventRecord(ev[2 * kBatch + 1], s));
            hipLaunchKernelGGL(kh_cg_init, dim3(1), dim3(1024), 0, s, part, nb, cs, prtol, pcgmax);
            HIP_TRY(hipGetLastError());
            HCg c;
            HIP_TRY(hipMemcpyAsync(&c, cs, sizeof(c), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (tk) {
                H->kt_ms[2] += elapsed(2 * kBatch, 2 * kBatch + 1);
                H->kt_calls[2] += 1;
            }
            gnorm = c.gmax;
            if (!is_fin(gnorm)) return L1LS_E_NONFINITE;
            if (gnorm <= gtol) {
                converged = true;
                break;
            }
            L1LS_TRY(pcg(c));
            double a = 0;
            L1LS_TRY(line_search(&a));
            hipLaunchKernelGGL(kh_step, dim3(nb), dim3(kHB), 0, s, K.n / 2, (double2*)x, (double2*)gd,
                               (const double2*)dx, a, mu, primal);
            HIP_TRY(hipGetLastError());
            ++newton;
        }
        HIP_TRY(hipStreamSynchronize(s));
        return L1LS_OK;
    }

    l1ls_status report(l1ls_report* out) {
        l1ls_report rr;
        std::memset(&rr, 0, sizeof(rr));
        rr.iterations = newton;
        rr.inner = pcg_total;
        L1LS_TRY(sgt_gap(H, tau, x, s, &rr.primal, &rr.dual, &rr.rel_gap, part));
        L1LS_TRY(sgt_err(H, x, s, &rr.rel_err, part));
        rr.converged = converged ? 1 : 0;
        rr.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (out) *out = rr;
        return L1LS_OK;
    }
};

extern "C" l1ls_status l1ls_sgt_newton_create(const l1ls_sgt* H, const l1ls_solve_opts* o, double* x,
                                               l1ls_sgt_newton** out) {
    if (!H || !o || !x || !out) return L1LS_E_ARG;
    *out = nullptr;
    if (!aligned16(x) || (o->x0_dev && !aligned16(o->x0_dev))) return L1LS_E_ARG;
    if (o->precision != L1LS_F64 || o->polish != 0) return L1LS_E_UNSUPPORTED;
    auto* N = new (std::nothrow) l1ls_sgt_newton();
    if (!N) return L1LS_E_NOMEM;
    const l1ls_status st = N->init(H, o, x);
    if (st != L1LS_OK) {
        delete N;
        return st;
    }
    *out = N;
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_sgt_newton_step(l1ls_sgt_newton* N, int64_t steps, l1ls_report* rep) {
    if (!N || steps < 0) return L1LS_E_ARG;
    L1LS_TRY(N->steps(steps));
    L1LS_TRY(N->report(rep));
    return N->converged ? L1LS_OK : L1LS_NOT_CONVERGED;
}

extern "C" void l1ls_sgt_newton_destroy(l1ls_sgt_newton* N) { delete N; }

extern "C" l1ls_status l1ls_sgt_solve_cg_newton(const l1ls_sgt* H, const l1ls_solve_opts* o, double* x,
                                                 l1ls_report* rep) {
    if (!H || !o || !x) return L1LS_E_ARG;
    if (o->max_iter < 0) return L1LS_E_ARG;
    l1ls_sgt_newton* N = nullptr;
    L1LS_TRY(l1ls_sgt_newton_create(H, o, x, &N));
    const l1ls_status st = l1ls_sgt_newton_step(N, o->max_iter, rep);
    l1ls_sgt_newton_destroy(N);
    return st;
}

extern "C" l1ls_status l1ls_sgt_kernel_times(const l1ls_sgt* H, double* ms, int64_t* calls) {
    if (!H || !ms || !calls) return L1LS_E_ARG;
    for (int q = 0; q < 3; ++q) {
        ms[q] = H->kt_ms[q];
        calls[q] = H->kt_calls[q];
    }
    return L1LS_OK;
}
