// Procedure IGen2 (section 3.2): instances with fewer rows than columns.
//
// The procedure takes B (m x m, rank m), N (m x (n - m)) and x* with its
// support among B's columns; it sets e = tau B^{-T} g for a subgradient g of
// x*'s first m components (step 3), rescales every column of N to
// N~_k = xi_k tau / |N_k^T e| N_k with xi_k in [-1, 1] (step 4), and returns
// A = [B, N~], b = A x* + e.  Here:
//   * B, x*, g and e are those of the generator's square instance (m x m,
//     one rotation stage per side): B^{-T} = Q Sigma^{-1} G^T is what IGen's
//     step 3 already applies, so the square instance is built first and
//     extended in place;
//   * column k of N is a copy of column p(k) of B, p injective, drawn among
//     the columns j with |g_j| >= 1/2 (positions 0 .. n-m-1 of a random
//     bijection of that list), so N_k^T e = tau g_p and the scale
//     |xi_k| / |g_p| stays <= 2;
//   * x* is zero on N~, so b is B's; A^T e = tau g with g_{m+k} =
//     xi_k sign(N_k^T e), and x* is optimal (eq. (15)).
//   * L = 1 + max_k c_k^2 bounds lambda_max(A A^T) = lambda_max(B (I +
//     P D^2 P^T) B^T) with sigma_1 = 1 (P D the placement and scales of N~).
// The N~ columns follow B's in operator order (position m + k is original
// column m + k).  A row of B has at most 4 entries at one stage and, p being
// injective, gains at most 4 from N~, so the stored kernels' limits hold.
#include <algorithm>
#include <cstdint>

#include "common.hpp"
#include "rng.hpp"

using namespace l1ls;

l1ls_status exclusive_scan_i32(const int32_t* counts, int32_t* offsets, int64_t n, hipStream_t stream,
                               DevArena& tmp);

namespace {

constexpr uint32_t kTagIgen2Pick = 0x900u;  // bijection of the eligible columns
constexpr uint32_t kTagIgen2Xi = 0xA00u;    // counter (k, 0, tag, 0): xi_k

inline dim3 g1d(int64_t N) { return dim3((unsigned)std::max<int64_t>(1, (N + L1LS_BLOCK - 1) / L1LS_BLOCK)); }

__global__ void k_elig_flag(const double* __restrict__ g, int64_t m, int32_t* __restrict__ flag) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) flag[j] = fabs(g[j]) >= 0.5 ? 1 : 0;
}

__global__ void k_elig_list(const int32_t* __restrict__ flag, const int32_t* __restrict__ off, int64_t m,
                            int32_t* __restrict__ list) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m && flag[j]) list[off[j]] = (int32_t)j;
}

// p_k, xi_k; inv[position of p_k] = k.
__global__ void k_pick(const int32_t* __restrict__ list, int64_t count, int64_t nn, Key key,
                       const int32_t* __restrict__ col_pos, int32_t* __restrict__ ppos, double* __restrict__ xi,
                       int32_t* __restrict__ inv) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    const int32_t p = list[bijection(k, count, kTagIgen2Pick, key)];
    const int32_t q = col_pos ? col_pos[p] : p;
    ppos[k] = q;
    inv[q] = (int32_t)k;
    const U4 w = philox4x32_10((uint32_t)k, 0u, kTagIgen2Xi, 0u, key.k0, key.k1);
    xi[k] = __dadd_rn(__dmul_rn(2.0, unit_double(w.x, w.y)), -1.0);
}

// c_k = xi_k tau / |N_k^T e| with N_k B's stored column at position ppos[k];
// g_{m+k} = xi_k sign(N_k^T e); cnt[k] = the column's entries.
__global__ void k_scales(const int32_t* __restrict__ ptr, const int32_t* __restrict__ row,
                         const double* __restrict__ v, const double* __restrict__ e_op,
                         const int32_t* __restrict__ ppos, const double* __restrict__ xi, double tau, int64_t nn,
                         double* __restrict__ c, double* __restrict__ gN, int32_t* __restrict__ cnt) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    const int32_t q = ppos[k];
    double d = 0.0;
    for (int32_t t = ptr[q]; t < ptr[q + 1]; ++t) d = __dadd_rn(d, __dmul_rn(v[t], e_op[row[t]]));
    c[k] = xi[k] * tau / fabs(d);
    gN[k] = d > 0.0 ? xi[k] : -xi[k];
    cnt[k] = ptr[q + 1] - ptr[q];
}

// The N~ columns of the new CSC (after B's nnz0 entries), and their squared
// norms (colnorm2 at position m + k).
__global__ void k_csc_n(const int32_t* __restrict__ ptr, const int32_t* __restrict__ row,
                        const double* __restrict__ v, const int32_t* __restrict__ ppos, const double* __restrict__ c,
                        const int32_t* __restrict__ off, int32_t nnz0, int64_t nn, int32_t* __restrict__ row2,
                        double* __restrict__ v2, int32_t* __restrict__ ptr2_tail, double* __restrict__ cn2) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nn) return;
    const int32_t q = ppos[k];
    int32_t o = nnz0 + off[k];
    double s = 0.0;
    for (int32_t t = ptr[q]; t < ptr[q + 1]; ++t, ++o) {
        const double a = c[k] * v[t];
        row2[o] = row[t];
        v2[o] = a;
        s += a * a;
    }
    ptr2_tail[k] = nnz0 + off[k + 1];
    cn2[k] = s;
}

// Row counts of the new CSR: B's entries plus one per entry whose column N~
// copies.
__global__ void k_csr_count2(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                             const int32_t* __restrict__ inv, int64_t m, int32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int32_t c = 0;
    for (int32_t t = ptr[i]; t < ptr[i + 1]; ++t) c += 1 + (inv[col[t]] >= 0 ? 1 : 0);
    cnt[i] = c;
}

// Row i of the new CSR: B's entries, then the N~ entries in column order.
__global__ void k_csr_fill2(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                            const double* __restrict__ v, const int32_t* __restrict__ inv,
                            const double* __restrict__ c, const int32_t* __restrict__ ptr2, int64_t m,
                            int32_t* __restrict__ col2, double* __restrict__ v2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int32_t o = ptr2[i];
    for (int32_t t = ptr[i]; t < ptr[i + 1]; ++t, ++o) {
        col2[o] = col[t];
        v2[o] = v[t];
    }
    const int32_t first = o;
    for (int32_t t = ptr[i]; t < ptr[i + 1]; ++t) {
        const int32_t k = inv[col[t]];
        if (k < 0) continue;
        // insertion into the sorted tail [first, o)
        int32_t u = o++;
        const int32_t cj = (int32_t)(m + k);
        const double a = c[k] * v[t];
        while (u > first && col2[u - 1] > cj) {
            col2[u] = col2[u - 1];
            v2[u] = v2[u - 1];
            --u;
        }
        col2[u] = cj;
        v2[u] = a;
    }
}

__global__ void k_ext_perm(const int32_t* __restrict__ old, int64_t m, int64_t n, int32_t* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) out[j] = j < m ? (old ? old[j] : (int32_t)j) : (int32_t)j;
}

__global__ void k_ext_vec(const double* __restrict__ old, int64_t m, const double* __restrict__ tail, int64_t n,
                          double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) out[j] = j < m ? old[j] : (tail ? tail[j - m] : 0.0);
}

__global__ void k_f64_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) b[i] = (float)a[i];
}

__global__ void k_max_sq(const double* __restrict__ c, int64_t N, double* __restrict__ out) {
    __shared__ double red[1024];
    double v = 0.0;
    for (int64_t k = threadIdx.x; k < N; k += blockDim.x) v = fmax(v, c[k] * c[k]);
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

}  // namespace

// Extend the square instance I (m x m, one stage, stored FP64 CSR/CSC) to
// IGen2's m x n instance in place.  L1LS_E_ARG when n - m exceeds the
// columns of B eligible for N (those with |g_j| >= 1/2).
l1ls_status igen2_extend(l1ls_instance* I, int64_t n, hipStream_t s) {
    const int64_t m = I->m, nn = n - m;
    if (I->n != m || nn < 1 || !I->csr_v64 || !I->csc_v64) return L1LS_E_ARG;
    const int32_t nnz0 = (int32_t)I->nnz;
    DevArena tmp;
    tmp.al = I->arena.al;
    auto fail = [&](l1ls_status st) {
        (void)hipStreamSynchronize(s);
        tmp.release();
        return st;
    };
    l1ls_status st;
    int32_t *flag = nullptr, *off = nullptr, *list = nullptr;
    if ((st = tmp.alloc(&flag, m)) != L1LS_OK) return fail(st);
    if ((st = tmp.alloc(&off, m + 1)) != L1LS_OK) return fail(st);
    if ((st = tmp.alloc(&list, m)) != L1LS_OK) return fail(st);
    hipLaunchKernelGGL(k_elig_flag, g1d(m), dim3(L1LS_BLOCK), 0, s, (const double*)I->g, m, flag);
    if ((st = exclusive_scan_i32(flag, off, m, s, tmp)) != L1LS_OK) return fail(st);
    int32_t count = 0;
    if (hipMemcpyAsync(&count, off + m, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(L1LS_E_HIP);
    if (nn > count) return fail(L1LS_E_ARG);
    hipLaunchKernelGGL(k_elig_list, g1d(m), dim3(L1LS_BLOCK), 0, s, (const int32_t*)flag, (const int32_t*)off, m,
                       list);
    // picks, scales and the new CSC
    int32_t *ppos = nullptr, *inv = nullptr, *cnt = nullptr, *coff = nullptr;
    double *xi = nullptr, *c = nullptr, *gN = nullptr, *e_op = nullptr, *cn2 = nullptr, *mx = nullptr;
    if ((st = tmp.alloc(&ppos, nn)) != L1LS_OK || (st = tmp.alloc(&inv, m)) != L1LS_OK ||
        (st = tmp.alloc(&cnt, nn)) != L1LS_OK || (st = tmp.alloc(&coff, nn + 1)) != L1LS_OK ||
        (st = tmp.alloc(&xi, nn)) != L1LS_OK || (st = tmp.alloc(&c, nn)) != L1LS_OK ||
        (st = tmp.alloc(&gN, nn)) != L1LS_OK || (st = tmp.alloc(&e_op, m)) != L1LS_OK ||
        (st = tmp.alloc(&cn2, nn)) != L1LS_OK || (st = tmp.alloc(&mx, 1)) != L1LS_OK)
        return fail(st);
    if (hipMemsetAsync(inv, 0xff, m * sizeof(int32_t), s) != hipSuccess) return fail(L1LS_E_HIP);
    const Key key = seed_key(I->seed);
    hipLaunchKernelGGL(k_pick, g1d(nn), dim3(L1LS_BLOCK), 0, s, (const int32_t*)list, (int64_t)count, nn, key,
                       I->op_col_pos, ppos, xi, inv);
    hipLaunchKernelGGL((k_gather_perm<double, double>), g1d(m), dim3(L1LS_BLOCK), 0, s, (const double*)I->e, e_op,
                       I->op_row_of, m);
    hipLaunchKernelGGL(k_scales, g1d(nn), dim3(L1LS_BLOCK), 0, s, (const int32_t*)I->csc_ptr,
                       (const int32_t*)I->csc_row, (const double*)I->csc_v64, (const double*)e_op,
                       (const int32_t*)ppos, (const double*)xi, I->tau, nn, c, gN, cnt);
    if ((st = exclusive_scan_i32(cnt, coff, nn, s, tmp)) != L1LS_OK) return fail(st);
    int32_t addc = 0;
    if (hipMemcpyAsync(&addc, coff + nn, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(L1LS_E_HIP);
    const int64_t nnz2 = (int64_t)nnz0 + addc;
    if (nnz2 >= ((int64_t)1 << 31)) return fail(L1LS_E_UNSUPPORTED);
    int32_t *cptr2 = nullptr, *crow2 = nullptr, *rptr2 = nullptr, *rcol2 = nullptr, *rcnt = nullptr;
    double *cv2 = nullptr, *rv2 = nullptr;
    if ((st = I->arena.alloc(&cptr2, n + 1)) != L1LS_OK || (st = I->arena.alloc(&crow2, nnz2)) != L1LS_OK ||
        (st = I->arena.alloc(&cv2, nnz2)) != L1LS_OK || (st = I->arena.alloc(&rptr2, m + 1)) != L1LS_OK ||
        (st = I->arena.alloc(&rcol2, nnz2)) != L1LS_OK || (st = I->arena.alloc(&rv2, nnz2)) != L1LS_OK ||
        (st = tmp.alloc(&rcnt, m)) != L1LS_OK)
        return fail(st);
    if (hipMemcpyAsync(cptr2, I->csc_ptr, (m + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(crow2, I->csc_row, (size_t)nnz0 * sizeof(int32_t), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(cv2, I->csc_v64, (size_t)nnz0 * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(L1LS_E_HIP);
    hipLaunchKernelGGL(k_csc_n, g1d(nn), dim3(L1LS_BLOCK), 0, s, (const int32_t*)I->csc_ptr,
                       (const int32_t*)I->csc_row, (const double*)I->csc_v64, (const int32_t*)ppos, (const double*)c,
                       (const int32_t*)coff, nnz0, nn, crow2, cv2, cptr2 + m + 1, cn2);
    // the new CSR
    hipLaunchKernelGGL(k_csr_count2, g1d(m), dim3(L1LS_BLOCK), 0, s, (const int32_t*)I->csr_ptr,
                       (const int32_t*)I->csr_col, (const int32_t*)inv, m, rcnt);
    if ((st = exclusive_scan_i32(rcnt, rptr2, m, s, tmp)) != L1LS_OK) return fail(st);
    hipLaunchKernelGGL(k_csr_fill2, g1d(m), dim3(L1LS_BLOCK), 0, s, (const int32_t*)I->csr_ptr,
                       (const int32_t*)I->csr_col, (const double*)I->csr_v64, (const int32_t*)inv, (const double*)c,
                       (const int32_t*)rptr2, m, rcol2, rv2);
    // vectors of length n
    int32_t *colof = nullptr, *colpos = nullptr;
    double *xs2 = nullptr, *g2 = nullptr, *cn = nullptr, *cnop = nullptr;
    if ((st = I->arena.alloc(&colof, n)) != L1LS_OK || (st = I->arena.alloc(&colpos, n)) != L1LS_OK ||
        (st = I->arena.alloc(&xs2, n)) != L1LS_OK || (st = I->arena.alloc(&g2, n)) != L1LS_OK ||
        (st = I->arena.alloc(&cn, n)) != L1LS_OK || (st = I->arena.alloc(&cnop, n)) != L1LS_OK)
        return fail(st);
    hipLaunchKernelGGL(k_ext_perm, g1d(n), dim3(L1LS_BLOCK), 0, s, I->op_col_of, m, n, colof);
    hipLaunchKernelGGL(k_ext_perm, g1d(n), dim3(L1LS_BLOCK), 0, s, I->op_col_pos, m, n, colpos);
    hipLaunchKernelGGL(k_ext_vec, g1d(n), dim3(L1LS_BLOCK), 0, s, (const double*)I->xstar, m, (const double*)nullptr,
                       n, xs2);
    hipLaunchKernelGGL(k_ext_vec, g1d(n), dim3(L1LS_BLOCK), 0, s, (const double*)I->g, m, (const double*)gN, n, g2);
    hipLaunchKernelGGL(k_ext_vec, g1d(n), dim3(L1LS_BLOCK), 0, s, (const double*)I->colnorm2, m, (const double*)cn2,
                       n, cn);
    hipLaunchKernelGGL(k_ext_vec, g1d(n), dim3(L1LS_BLOCK), 0, s, (const double*)I->colnorm2_op, m,
                       (const double*)cn2, n, cnop);
    hipLaunchKernelGGL(k_max_sq, dim3(1), dim3(1024), 0, s, (const double*)c, nn, mx);
    float *cv32 = nullptr, *rv32 = nullptr;
    const bool f32 = (I->storage & L1LS_STORE_F32) != 0;
    if (f32) {
        if ((st = I->arena.alloc(&cv32, nnz2)) != L1LS_OK || (st = I->arena.alloc(&rv32, nnz2)) != L1LS_OK)
            return fail(st);
        hipLaunchKernelGGL(k_f64_to_f32, g1d(nnz2), dim3(L1LS_BLOCK), 0, s, (const double*)cv2, cv32, nnz2);
        hipLaunchKernelGGL(k_f64_to_f32, g1d(nnz2), dim3(L1LS_BLOCK), 0, s, (const double*)rv2, rv32, nnz2);
    }
    double maxc2 = 0.0;
    int32_t rnnz = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&maxc2, mx, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&rnnz, rptr2 + m, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(L1LS_E_HIP);
    if (rnnz != nnz2) return fail(L1LS_E_STATE);
    tmp.release();
    // the square instance's stores and vectors of length m give way
    for (void* old : {(void*)I->csr_ptr, (void*)I->csr_col, (void*)I->csr_v64, (void*)I->csr_v32,
                      (void*)I->csc_ptr, (void*)I->csc_row, (void*)I->csc_v64, (void*)I->csc_v32, (void*)I->xstar,
                      (void*)I->g, (void*)I->colnorm2, (void*)I->colnorm2_op})
        I->arena.free_one(old);
    I->csc_ptr = cptr2;
    I->csc_row = crow2;
    I->csc_v64 = cv2;
    I->csc_v32 = cv32;
    I->csr_ptr = rptr2;
    I->csr_col = rcol2;
    I->csr_v64 = rv2;
    I->csr_v32 = rv32;
    I->op_col_of = colof;
    I->op_col_pos = colpos;
    I->xstar = xs2;
    I->g = g2;
    I->colnorm2 = cn;
    I->colnorm2_op = cnop;
    I->n = n;
    I->nnz = nnz2;
    I->L = 1.0 + maxc2;
    I->igen2 = true;
    // A = [B, N~] has no rotation form: the matrix-free operator is off
    I->mf_emb = nullptr;
    return L1LS_OK;
}
