// Instance generator on the GPU: Procedure IGen (section 3.1) with the
// SVD-known A = Q Sigma G^T of eq. (16) (section 4), the sparsity stages of
// section 4.2 and an OsGen-style x* (section 6).  Builds the pair tables,
// x*, the subgradient g, e, b, f* and the stored CSR/CSC (FP32 + FP64).
#include <cmath>

#include "common.hpp"
#include "rng.hpp"
#include "stages.hpp"

using namespace l1ls;

namespace {

__global__ void k_bijection(int32_t* __restrict__ perm, int32_t* __restrict__ pinv, int64_t N,
                            uint32_t tag, Key key) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    const int64_t y = bijection(a, N, tag, key);
    perm[a] = (int32_t)y;
    pinv[y] = (int32_t)a;
}

__global__ void k_support(int32_t* __restrict__ support, int64_t s, int64_t n, Key key) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= s) return;
    support[q] = (int32_t)bijection(q, n, kTagPerm | 2u, key);
}

__global__ void k_angles(double* __restrict__ cs, int64_t npairs, int side, int t, Key key) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npairs) return;
    double c, s;
    rotation_angle(side, t, (uint32_t)k, key, &c, &s);
    cs[2 * k] = c;
    cs[2 * k + 1] = s;
}

// sigma_j = kappa^(-(j-1)/(n-1)) (1-based j; 0-based here)
__global__ void k_sigma(double* __restrict__ sigma, int64_t n, double kappa) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    sigma[j] = pow(kappa, -__ddiv_rn((double)j, (double)(n - 1)));
}

// g_i = 0.9 (2u - 1), u from counter (i, 0, kTagSubgrad, 0); x* = 0.
__global__ void k_subgrad(double* __restrict__ g, double* __restrict__ xstar, int64_t n, Key key) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const U4 w = philox4x32_10((uint32_t)i, 0u, kTagSubgrad, 0u, key.k0, key.k1);
    g[i] = __dmul_rn(0.9, __dadd_rn(__dmul_rn(2.0, unit_double(w.x, w.y)), -1.0));
    xstar[i] = 0.0;
}

// x*_{support[q]} ~ N(0,1) by Box-Muller from counter (q, 0, kTagXstar, 0);
// g = sign(x*) on the support (eq. (10)).
__global__ void k_xstar(const int32_t* __restrict__ support, double* __restrict__ xstar,
                        double* __restrict__ g, int64_t s, Key key) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= s) return;
    const U4 w = philox4x32_10((uint32_t)q, 0u, kTagXstar, 0u, key.k0, key.k1);
    const double u1 = unit_double(w.x, w.y);
    const double u2 = unit_double(w.z, w.w);
    const double rad = sqrt(__dmul_rn(-2.0, log(__dsub_rn(1.0, u1))));
    const double z = __dmul_rn(rad, cos(__dmul_rn(2.0 * M_PI, u2)));
    const int32_t i = support[q];
    xstar[i] = z;
    g[i] = (z > 0.0) ? 1.0 : ((z < 0.0) ? -1.0 : 0.0);
}

template <typename T>
__global__ void k_stage(const T* __restrict__ in, T* __restrict__ out, SideTables tab, int t,
                        int transpose) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tab.N) return;
    const PairRef p = pair_of(tab, t, (int32_t)i);
    out[i] = stage_elem<T>(p, in[i], in[p.partner], transpose != 0);
}

// z (m) from w (n): mode 0: z_k = sigma_k w_k; mode 1: z_k = (tau w_k)/sigma_k;
// z_k = 0 for k >= n.
__global__ void k_embed(const double* __restrict__ w, double* __restrict__ z,
                        const double* __restrict__ sigma, int64_t n, int64_t m, int mode, double tau) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    if (k >= n) {
        z[k] = 0.0;
        return;
    }
    z[k] = (mode == 0) ? __dmul_rn(sigma[k], w[k]) : __ddiv_rn(__dmul_rn(tau, w[k]), sigma[k]);
}

__global__ void k_add(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out,
                      int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    out[i] = __dadd_rn(a[i], b[i]);
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ out, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    out[i] = (float)a[i];
}

// Per-block partial sums of |x| (stat 0) and e^2 (stat 1).
__global__ void k_fstar_partials(const double* __restrict__ x, int64_t n, const double* __restrict__ e,
                                 int64_t m, double* __restrict__ partials) {
    double v[2] = {0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        if (i < n) v[0] += fabs(x[i]);
        v[1] += e[i] * e[i];
    }
    block_reduce_stats<2, 2>(v);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = v[0];
        partials[2 * blockIdx.x + 1] = v[1];
    }
}

// ||A e_j||^2 = ||Sigma G^T e_j||^2 (Q is orthogonal): diag(A^T A) from the
// n-side stages alone.
template <int MAXE>
__global__ void k_colnorm(SideTables Gs, int rounds, const double* __restrict__ sigma, int64_t n,
                          double* __restrict__ colnorm2) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    SparseVec<MAXE> a, b;
    a.cnt = 1;
    a.idx[0] = (int32_t)j;
    a.val[0] = 1.0;
    SparseVec<MAXE>* cur = &a;
    SparseVec<MAXE>* nxt = &b;
    for (int t = rounds; t >= 1; --t) {
        stage_sparse(Gs, t, true, *cur, *nxt);
        SparseVec<MAXE>* tmp = cur; cur = nxt; nxt = tmp;
    }
    double acc = 0.0;
    for (int e = 0; e < cur->cnt; ++e) {
        const double v = __dmul_rn(sigma[cur->idx[e]], cur->val[e]);
        acc = __dadd_rn(acc, __dmul_rn(v, v));
    }
    colnorm2[j] = acc;
}

// Column at operator position c (original column col_of[c]); row indices
// mapped to operator positions row_pos[i] and sorted.
template <int MAXE>
__device__ __forceinline__ void op_column(SideTables Gs, SideTables Qs, int rounds, const double* sigma,
                                          const int32_t* col_of, const int32_t* row_pos, int64_t c,
                                          SparseVec<MAXE>& col) {
    const int32_t j = col_of ? col_of[c] : (int32_t)c;
    column_of_A<MAXE>(Gs, Qs, rounds, sigma, j, col);
    if (row_pos) {
        for (int e = 0; e < col.cnt; ++e) col.idx[e] = row_pos[col.idx[e]];
        sort_sparse(col);
    }
}

template <int MAXE>
__global__ void k_csc_count(SideTables Gs, SideTables Qs, int rounds, const double* __restrict__ sigma,
                            int64_t n, int32_t* __restrict__ counts) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    SparseVec<MAXE> col;
    column_of_A<MAXE>(Gs, Qs, rounds, sigma, (int32_t)j, col);
    counts[j] = col.cnt;
}

template <int MAXE>
__global__ void k_csc_fill(SideTables Gs, SideTables Qs, int rounds, const double* __restrict__ sigma,
                           int64_t n, const int32_t* __restrict__ col_of, const int32_t* __restrict__ row_pos,
                           const int32_t* __restrict__ ptr, int32_t* __restrict__ row, double* __restrict__ val) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    SparseVec<MAXE> col;
    op_column<MAXE>(Gs, Qs, rounds, sigma, col_of, row_pos, c, col);
    const int32_t base = ptr[c];
    for (int e = 0; e < col.cnt; ++e) {
        row[base + e] = col.idx[e];
        val[base + e] = col.val[e];
    }
}

template <int MAXE>
__device__ __forceinline__ void op_row(SideTables Gs, SideTables Qs, int rounds, int64_t n, const double* sigma,
                                       const int32_t* row_of, const int32_t* col_pos, int64_t p,
                                       SparseVec<MAXE>& r) {
    const int32_t i = row_of ? row_of[p] : (int32_t)p;
    row_pattern_of_A<MAXE>(Gs, Qs, rounds, n, sigma, i, r);
    if (col_pos) {
        for (int e = 0; e < r.cnt; ++e) r.idx[e] = col_pos[r.idx[e]];
        sort_sparse(r);
    }
}

template <int MAXE>
__global__ void k_csr_count(SideTables Gs, SideTables Qs, int rounds, const double* __restrict__ sigma,
                            int64_t n, int64_t m, int32_t* __restrict__ counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    SparseVec<MAXE> r;
    row_pattern_of_A<MAXE>(Gs, Qs, rounds, n, sigma, (int32_t)i, r);
    counts[i] = r.cnt;
}

// counts in operator order: cnt_op[p] = cnt[of[p]]
__global__ void k_perm_counts(const int32_t* __restrict__ cnt, int32_t* __restrict__ out,
                              const int32_t* __restrict__ of, int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    out[p] = cnt[of ? of[p] : p];
}

// Row i gets its values from the stored columns, so CSR and CSC hold the
// same numbers bit for bit.
template <int MAXE>
__global__ void k_csr_fill(SideTables Gs, SideTables Qs, int rounds, const double* __restrict__ sigma,
                           int64_t n, int64_t m, const int32_t* __restrict__ row_of,
                           const int32_t* __restrict__ col_pos, const int32_t* __restrict__ ptr,
                           int32_t* __restrict__ col, double* __restrict__ val, const int32_t* __restrict__ csc_ptr,
                           const int32_t* __restrict__ csc_row, const double* __restrict__ csc_val,
                           int32_t* __restrict__ missing) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    SparseVec<MAXE> r;
    op_row<MAXE>(Gs, Qs, rounds, n, sigma, row_of, col_pos, i, r);
    const int32_t base = ptr[i];
    for (int e = 0; e < r.cnt; ++e) {
        const int32_t j = r.idx[e];
        double v = 0.0;
        bool found = false;
        for (int32_t q = csc_ptr[j]; q < csc_ptr[j + 1]; ++q)
            if (csc_row[q] == (int32_t)i) {
                v = csc_val[q];
                found = true;
                break;
            }
        if (!found) atomicAdd(missing, 1);
        col[base + e] = j;
        val[base + e] = v;
    }
}

// --- exclusive scan (three passes) -----------------------------------------
constexpr int kScanItems = 8;

__global__ void k_scan_local(const int32_t* __restrict__ in, int32_t* __restrict__ out, int64_t n,
                             int64_t* __restrict__ block_tot) {
    __shared__ int64_t sh[L1LS_BLOCK];
    const int64_t base = (int64_t)blockIdx.x * L1LS_BLOCK * kScanItems + threadIdx.x * kScanItems;
    int64_t loc[kScanItems];
    int64_t acc = 0;
    for (int q = 0; q < kScanItems; ++q) {
        loc[q] = acc;
        acc += (base + q < n) ? in[base + q] : 0;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 1; o < L1LS_BLOCK; o <<= 1) {
        const int64_t v = (threadIdx.x >= (unsigned)o) ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    const int64_t excl = sh[threadIdx.x] - acc;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < n) out[base + q] = (int32_t)(excl + loc[q]);
    if (threadIdx.x == L1LS_BLOCK - 1) block_tot[blockIdx.x] = sh[threadIdx.x];
}

__global__ void k_scan_totals(int64_t* __restrict__ tot, int64_t nblocks) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t acc = 0;
    for (int64_t b = 0; b < nblocks; ++b) {
        const int64_t v = tot[b];
        tot[b] = acc;
        acc += v;
    }
    tot[nblocks] = acc;
}

__global__ void k_scan_add(int32_t* __restrict__ out, int64_t n, const int64_t* __restrict__ tot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += (int32_t)tot[i / (L1LS_BLOCK * kScanItems)];
    if (i == n) out[n] = (int32_t)tot[(n + L1LS_BLOCK * kScanItems - 1) / (L1LS_BLOCK * kScanItems)];
}

inline dim3 grid1(int64_t N) { return dim3((unsigned)((N + L1LS_BLOCK - 1) / L1LS_BLOCK)); }

}  // namespace

l1ls_status exclusive_scan_i32(const int32_t* counts, int32_t* offsets, int64_t n, hipStream_t stream,
                               DevArena& tmp) {
    const int64_t per = (int64_t)L1LS_BLOCK * kScanItems;
    const int64_t nb = (n + per - 1) / per;
    int64_t* tot = nullptr;
    L1LS_TRY(tmp.alloc(&tot, nb + 1));
    hipLaunchKernelGGL(k_scan_local, dim3((unsigned)std::max<int64_t>(nb, 1)), dim3(L1LS_BLOCK), 0, stream,
                       counts, offsets, n, tot);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1), 0, stream, tot, nb);
    hipLaunchKernelGGL(k_scan_add, grid1(n + 1), dim3(L1LS_BLOCK), 0, stream, offsets, n, tot);
    HIP_TRY(hipGetLastError());
    return L1LS_OK;
}

// Apply G^T (stage r first) or G (stage 1 first), or Q / Q^T, to a device
// vector, ping-ponging between `v` and `scratch`; the result ends in `v`.
template <typename T>
l1ls_status apply_side(const SideTables& tab, int rounds, bool transpose, T* v, T* scratch,
                       hipStream_t stream) {
    for (int q = 0; q < rounds; ++q) {
        const int t = transpose ? rounds - q : q + 1;
        hipLaunchKernelGGL(k_stage<T>, grid1(tab.N), dim3(L1LS_BLOCK), 0, stream, v, scratch, tab, t,
                           transpose ? 1 : 0);
        HIP_TRY(hipMemcpyAsync(v, scratch, tab.N * sizeof(T), hipMemcpyDeviceToDevice, stream));
    }
    HIP_TRY(hipGetLastError());
    return L1LS_OK;
}
template l1ls_status apply_side<double>(const SideTables&, int, bool, double*, double*, hipStream_t);
template l1ls_status apply_side<float>(const SideTables&, int, bool, float*, float*, hipStream_t);

l1ls_status build_mf_tables(l1ls_instance* I, hipStream_t s);
l1ls_status build_blocks(l1ls_instance* I, hipStream_t s, DevArena& tmp);
l1ls_status build_stored_windows(l1ls_instance* I, hipStream_t s);
l1ls_status igen2_extend(l1ls_instance* I, int64_t n, hipStream_t s);

// l1ls_generate_ex with the instance's device memory (and the build's
// temporaries) from `al` (nullptr: hipMalloc).
l1ls_status generate_with(int64_t m, int64_t n, double kappa, int64_t s, double tau, uint64_t seed,
                          const l1ls_gen_opts* opts, DevAlloc* al, l1ls_instance** out) {
    if (!out) return L1LS_E_ARG;
    *out = nullptr;
    const int rounds = opts ? opts->rounds : 1;
    const uint32_t storage = opts ? opts->storage : (L1LS_STORE_F32 | L1LS_STORE_F64);
    const int layout = opts ? opts->layout : L1LS_LAYOUT_STAGE;
    if (layout != L1LS_LAYOUT_NATURAL && layout != L1LS_LAYOUT_STAGE) return L1LS_E_ARG;
    hipStream_t stream = opts ? (hipStream_t)opts->stream : nullptr;
    if (m < n) {
        // Procedure IGen2 (section 3.2): the square instance B (m x m, one
        // stage), extended in place by the rescaled columns N~ (igen2.hip)
        if (!(m >= 2 && (m % 2) == 0 && n < ((int64_t)1 << 31))) return L1LS_E_ARG;
        if (!(s >= 0 && s <= m)) return L1LS_E_ARG;
        if (rounds != 1 || !(storage & (L1LS_STORE_F32 | L1LS_STORE_F64)) ||
            (storage & (L1LS_STORE_BLK32 | L1LS_STORE_MF_WINDOWS)))
            return L1LS_E_UNSUPPORTED;
        l1ls_gen_opts o2;
        o2.rounds = 1;
        o2.storage = (storage | L1LS_STORE_F64) & ~L1LS_STORE_WINDOWS;
        o2.stream = stream;
        o2.layout = layout;
        l1ls_instance* J = nullptr;
        L1LS_TRY(generate_with(m, m, kappa, s, tau, seed, &o2, al, &J));
        l1ls_status st = igen2_extend(J, n, stream);
        J->storage = storage | L1LS_STORE_F64;
        if (st == L1LS_OK && (storage & L1LS_STORE_WINDOWS)) st = build_stored_windows(J, stream);
        if (st != L1LS_OK) {
            (void)hipStreamSynchronize(stream);
            J->arena.release();
            delete J;
            return st;
        }
        *out = J;
        return L1LS_OK;
    }
    if (!(n >= 2 && m >= n && (m % 2) == 0 && (n % 2) == 0 && m < ((int64_t)1 << 31))) return L1LS_E_ARG;
    if (!(s >= 0 && s <= n) || !(kappa >= 1.0) || !is_finite(kappa) || !(tau > 0.0) || !is_finite(tau))
        return L1LS_E_ARG;
    if (rounds < 1 || rounds > L1LS_MAX_ROUNDS) return L1LS_E_ARG;
    if ((storage & ~(L1LS_STORE_F32 | L1LS_STORE_F64 | L1LS_STORE_BLK32 | L1LS_STORE_MF_WINDOWS |
                     L1LS_STORE_WINDOWS)) != 0)
        return L1LS_E_ARG;
    if ((storage & L1LS_STORE_BLK32) && (rounds != 2 || layout != L1LS_LAYOUT_STAGE || n < 4))
        return L1LS_E_UNSUPPORTED;
    if ((int64_t)16 * n >= ((int64_t)1 << 31) && (storage & (L1LS_STORE_F32 | L1LS_STORE_F64 | L1LS_STORE_BLK32)))
        return L1LS_E_UNSUPPORTED;
    // the stored passes gather FP64 vectors of m entries with 32-bit byte
    // offsets (below 4 GiB)
    if ((storage & (L1LS_STORE_F32 | L1LS_STORE_F64)) && m >= ((int64_t)1 << 29)) return L1LS_E_UNSUPPORTED;

    l1ls_instance* I = new l1ls_instance();
    I->m = m;
    I->n = n;
    I->s = s;
    I->kappa = kappa;
    I->tau = tau;
    I->seed = seed;
    I->rounds = rounds;
    I->storage = storage;
    I->layout = layout;
    I->L = 1.0;  // sigma_1 = kappa^0
    HIP_TRY(hipGetDevice(&I->device));
    I->arena.al = al;
    DevArena tmp;
    tmp.al = al;
    auto fail = [&](l1ls_status st) {
        (void)hipStreamSynchronize(stream);  // nothing queued may still use the buffers
        tmp.release();
        I->arena.release();
        delete I;
        return st;
    };
#define GEN_TRY(expr)                          \
    do {                                       \
        l1ls_status _s = (expr);               \
        if (_s != L1LS_OK) return fail(_s);    \
    } while (0)
#define GEN_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess) return fail(_e == hipErrorOutOfMemory ? L1LS_E_NOMEM : L1LS_E_HIP); \
    } while (0)

    const Key key = seed_key(seed);
    const int64_t Ns[2] = {n, m};
    for (int sd = 0; sd < 2; ++sd) {
        SideTables& T = I->side[sd];
        T.N = Ns[sd];
        GEN_TRY(I->arena.alloc(&T.perm, T.N));
        GEN_TRY(I->arena.alloc(&T.pinv, T.N));
        hipLaunchKernelGGL(k_bijection, grid1(T.N), dim3(L1LS_BLOCK), 0, stream, T.perm, T.pinv, T.N,
                           kTagPerm | (uint32_t)sd, key);
        for (int t = 1; t <= rounds; ++t) {
            GEN_TRY(I->arena.alloc(&T.cs[t - 1], T.N));
            hipLaunchKernelGGL(k_angles, grid1(T.N / 2), dim3(L1LS_BLOCK), 0, stream, T.cs[t - 1], T.N / 2,
                               sd, t, key);
        }
    }
    GEN_TRY(I->arena.alloc(&I->sigma, n));
    GEN_TRY(I->arena.alloc(&I->xstar, n));
    GEN_TRY(I->arena.alloc(&I->g, n));
    GEN_TRY(I->arena.alloc(&I->e, m));
    GEN_TRY(I->arena.alloc(&I->b, m));
    GEN_TRY(I->arena.alloc(&I->b32, m));
    GEN_TRY(I->arena.alloc(&I->support, s));
    GEN_TRY(I->arena.alloc(&I->colnorm2, n));
    hipLaunchKernelGGL(k_sigma, grid1(n), dim3(L1LS_BLOCK), 0, stream, I->sigma, n, kappa);
    hipLaunchKernelGGL(k_subgrad, grid1(n), dim3(L1LS_BLOCK), 0, stream, I->g, I->xstar, n, key);
    if (s > 0) {
        hipLaunchKernelGGL(k_support, grid1(s), dim3(L1LS_BLOCK), 0, stream, I->support, s, n, key);
        hipLaunchKernelGGL(k_xstar, grid1(s), dim3(L1LS_BLOCK), 0, stream, I->support, I->xstar, I->g, s, key);
    }
    GEN_HIP(hipGetLastError());

    // IGen step 3 with (A^T A)^{-1} = G (Sigma^T Sigma)^{-1} G^T:
    // e = tau Q Sigma^{+T} G^T g.  Step 4: b = A x* + e.
    double *wn = nullptr, *wn2 = nullptr, *zm = nullptr, *zm2 = nullptr;
    GEN_TRY(tmp.alloc(&wn, n));
    GEN_TRY(tmp.alloc(&wn2, n));
    GEN_TRY(tmp.alloc(&zm, m));
    GEN_TRY(tmp.alloc(&zm2, m));
    GEN_HIP(hipMemcpyAsync(wn, I->g, n * sizeof(double), hipMemcpyDeviceToDevice, stream));
    GEN_TRY(apply_side<double>(I->side[0], rounds, true, wn, wn2, stream));
    hipLaunchKernelGGL(k_embed, grid1(m), dim3(L1LS_BLOCK), 0, stream, wn, zm, I->sigma, n, m, 1, tau);
    GEN_TRY(apply_side<double>(I->side[1], rounds, false, zm, zm2, stream));
    GEN_HIP(hipMemcpyAsync(I->e, zm, m * sizeof(double), hipMemcpyDeviceToDevice, stream));
    GEN_HIP(hipMemcpyAsync(wn, I->xstar, n * sizeof(double), hipMemcpyDeviceToDevice, stream));
    GEN_TRY(apply_side<double>(I->side[0], rounds, true, wn, wn2, stream));
    hipLaunchKernelGGL(k_embed, grid1(m), dim3(L1LS_BLOCK), 0, stream, wn, zm, I->sigma, n, m, 0, tau);
    GEN_TRY(apply_side<double>(I->side[1], rounds, false, zm, zm2, stream));
    hipLaunchKernelGGL(k_add, grid1(m), dim3(L1LS_BLOCK), 0, stream, zm, I->e, I->b, m);
    hipLaunchKernelGGL(k_to_f32, grid1(m), dim3(L1LS_BLOCK), 0, stream, I->b, I->b32, m);
    GEN_HIP(hipGetLastError());

    // f* = tau ||x*||_1 + 0.5 ||e||^2
    const int nparts = 256;
    double* parts = nullptr;
    GEN_TRY(tmp.alloc(&parts, 2 * nparts));
    hipLaunchKernelGGL(k_fstar_partials, dim3(nparts), dim3(L1LS_BLOCK), 0, stream, I->xstar, n, I->e, m, parts);
    std::vector<double> hp(2 * nparts);
    GEN_HIP(hipMemcpyAsync(hp.data(), parts, hp.size() * sizeof(double), hipMemcpyDeviceToHost, stream));

    // diag(A^T A) for the preconditioners
    hipLaunchKernelGGL(k_colnorm<4>, grid1(n), dim3(L1LS_BLOCK), 0, stream, I->side[0], rounds, I->sigma, n,
                       I->colnorm2);
    // Column counts give nnz(A) whether or not A is stored.
    int32_t* counts = nullptr;
    int32_t* cptr = nullptr;
    GEN_TRY(tmp.alloc(&counts, m));
    GEN_TRY(((storage) ? I->arena : tmp).alloc(&cptr, n + 1));
    hipLaunchKernelGGL(k_csc_count<16>, grid1(n), dim3(L1LS_BLOCK), 0, stream, I->side[0], I->side[1], rounds,
                       I->sigma, n, counts);
    GEN_TRY(exclusive_scan_i32(counts, cptr, n, stream, tmp));
    int32_t nnz = 0;
    GEN_HIP(hipMemcpyAsync(&nnz, cptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    GEN_HIP(hipStreamSynchronize(stream));
    double fs[2] = {0.0, 0.0};
    for (int b = 0; b < nparts; ++b) {
        fs[0] += hp[2 * b];
        fs[1] += hp[2 * b + 1];
    }
    I->fstar = tau * fs[0] + 0.5 * fs[1];
    I->nnz = nnz;

    GEN_TRY(build_mf_tables(I, stream));

    // Operator order of the stored A and of the vectors that go with it.
    if (layout == L1LS_LAYOUT_STAGE) {
        I->op_col_of = I->side[0].perm;
        I->op_col_pos = I->side[0].pinv;
        I->op_row_of = I->side[1].perm;
        I->op_row_pos = I->side[1].pinv;
    }
    GEN_TRY(I->arena.alloc(&I->b_op, m));
    GEN_TRY(I->arena.alloc(&I->b32_op, m));
    GEN_TRY(I->arena.alloc(&I->colnorm2_op, n));
    hipLaunchKernelGGL((k_gather_perm<double, double>), grid1(m), dim3(L1LS_BLOCK), 0, stream, I->b, I->b_op,
                       I->op_row_of, m);
    hipLaunchKernelGGL((k_gather_perm<float, double>), grid1(m), dim3(L1LS_BLOCK), 0, stream, I->b, I->b32_op,
                       I->op_row_of, m);
    hipLaunchKernelGGL((k_gather_perm<double, double>), grid1(n), dim3(L1LS_BLOCK), 0, stream, I->colnorm2,
                       I->colnorm2_op, I->op_col_of, n);

    if (storage & L1LS_STORE_BLK32) GEN_TRY(build_blocks(I, stream, tmp));
    if (storage & (L1LS_STORE_F32 | L1LS_STORE_F64)) {
        // Stored CSC (columns A e_j) and CSR (rows A^T e_i) in operator order;
        // CSR values are looked up in the columns so both hold the same numbers.
        int32_t* cnt_op = nullptr;
        GEN_TRY(tmp.alloc(&cnt_op, m));
        if (I->op_col_of) {
            hipLaunchKernelGGL(k_perm_counts, grid1(n), dim3(L1LS_BLOCK), 0, stream, counts, cnt_op, I->op_col_of, n);
            GEN_TRY(exclusive_scan_i32(cnt_op, cptr, n, stream, tmp));
        }
        I->csc_ptr = cptr;
        double* csc_v64 = nullptr;
        GEN_TRY(I->arena.alloc(&I->csc_row, nnz));
        GEN_TRY(((storage & L1LS_STORE_F64) ? I->arena : tmp).alloc(&csc_v64, nnz));
        hipLaunchKernelGGL(k_csc_fill<16>, grid1(n), dim3(L1LS_BLOCK), 0, stream, I->side[0], I->side[1],
                           rounds, I->sigma, n, I->op_col_of, I->op_row_pos, I->csc_ptr, I->csc_row, csc_v64);
        GEN_TRY(I->arena.alloc(&I->csr_ptr, m + 1));
        hipLaunchKernelGGL(k_csr_count<16>, grid1(m), dim3(L1LS_BLOCK), 0, stream, I->side[0], I->side[1],
                           rounds, I->sigma, n, m, counts);
        if (I->op_row_of) {
            hipLaunchKernelGGL(k_perm_counts, grid1(m), dim3(L1LS_BLOCK), 0, stream, counts, cnt_op, I->op_row_of, m);
            GEN_TRY(exclusive_scan_i32(cnt_op, I->csr_ptr, m, stream, tmp));
        } else {
            GEN_TRY(exclusive_scan_i32(counts, I->csr_ptr, m, stream, tmp));
        }
        double* csr_v64 = nullptr;
        int32_t* missing = nullptr;
        GEN_TRY(tmp.alloc(&missing, 1));
        GEN_HIP(hipMemsetAsync(missing, 0, sizeof(int32_t), stream));
        GEN_TRY(I->arena.alloc(&I->csr_col, nnz));
        GEN_TRY(((storage & L1LS_STORE_F64) ? I->arena : tmp).alloc(&csr_v64, nnz));
        hipLaunchKernelGGL(k_csr_fill<16>, grid1(m), dim3(L1LS_BLOCK), 0, stream, I->side[0], I->side[1],
                           rounds, I->sigma, n, m, I->op_row_of, I->op_col_pos, I->csr_ptr, I->csr_col, csr_v64,
                           I->csc_ptr, I->csc_row, csc_v64, missing);
        if (storage & L1LS_STORE_F32) {
            GEN_TRY(I->arena.alloc(&I->csc_v32, nnz));
            GEN_TRY(I->arena.alloc(&I->csr_v32, nnz));
            hipLaunchKernelGGL(k_to_f32, grid1(nnz), dim3(L1LS_BLOCK), 0, stream, csc_v64, I->csc_v32,
                               (int64_t)nnz);
            hipLaunchKernelGGL(k_to_f32, grid1(nnz), dim3(L1LS_BLOCK), 0, stream, csr_v64, I->csr_v32,
                               (int64_t)nnz);
        }
        if (storage & L1LS_STORE_F64) {
            I->csc_v64 = csc_v64;
            I->csr_v64 = csr_v64;
        }
        int32_t miss = 0, csr_nnz = 0;
        GEN_HIP(hipMemcpyAsync(&miss, missing, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        GEN_HIP(hipMemcpyAsync(&csr_nnz, I->csr_ptr + m, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        GEN_HIP(hipGetLastError());
        GEN_HIP(hipStreamSynchronize(stream));
        if (miss != 0 || csr_nnz != nnz) {
            if (std::getenv("L1LS_DEBUG"))
                std::fprintf(stderr, "l1ls: CSR/CSC mismatch (missing %d, nnz %d vs %d)\n", miss, csr_nnz, nnz);
            return fail(L1LS_E_STATE);
        }
        if (storage & L1LS_STORE_WINDOWS) GEN_TRY(build_stored_windows(I, stream));
    }
    GEN_HIP(hipGetLastError());
    GEN_HIP(hipStreamSynchronize(stream));
    tmp.release();
    *out = I;
    return L1LS_OK;
#undef GEN_TRY
#undef GEN_HIP
}

extern "C" l1ls_status l1ls_generate(int64_t m, int64_t n, double kappa, int64_t s, double tau, uint64_t seed,
                                     l1ls_instance** out) {
    l1ls_gen_opts o;
    o.rounds = 1;
    o.storage = L1LS_STORE_F32 | L1LS_STORE_F64;
    o.stream = nullptr;
    o.layout = L1LS_LAYOUT_STAGE;
    return l1ls_generate_ex(m, n, kappa, s, tau, seed, &o, out);
}

extern "C" l1ls_status l1ls_instance_info(const l1ls_instance* I, l1ls_info* o) {
    if (!I || !o) return L1LS_E_ARG;
    o->m = I->m;
    o->n = I->n;
    o->s = I->s;
    o->nnz = I->nnz;
    o->rounds = I->rounds;
    o->storage = I->storage;
    o->layout = I->layout;
    o->kappa = I->kappa;
    o->tau = I->tau;
    o->L = I->L;
    o->f_star = I->fstar;
    o->seed = I->seed;
    o->b_dev = I->b;
    o->x_star_dev = I->xstar;
    o->g_dev = I->g;
    o->e_dev = I->e;
    o->sigma_dev = I->sigma;
    o->support_dev = I->support;
    o->perm_n_dev = I->side[0].perm;
    o->perm_m_dev = I->side[1].perm;
    for (int t = 0; t < 2; ++t) {
        o->cs_n_dev[t] = I->side[0].cs[t];
        o->cs_m_dev[t] = I->side[1].cs[t];
    }
    o->csr_ptr_dev = I->csr_ptr;
    o->csr_col_dev = I->csr_col;
    o->csr_val32_dev = I->csr_v32;
    o->csr_val64_dev = I->csr_v64;
    o->csc_ptr_dev = I->csc_ptr;
    o->csc_row_dev = I->csc_row;
    o->csc_val32_dev = I->csc_v32;
    o->csc_val64_dev = I->csc_v64;
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_generate_ex(int64_t m, int64_t n, double kappa, int64_t s, double tau,
                                        uint64_t seed, const l1ls_gen_opts* opts, l1ls_instance** out) {
    return generate_with(m, n, kappa, s, tau, seed, opts, nullptr, out);
}

// Free an instance whose device work has completed (the caller synchronised
// the streams that used it), without waiting for the rest of the device.
void free_idle_instance(l1ls_instance* I) {
    if (!I) return;
    I->arena.release();
    delete I;
}

extern "C" void l1ls_free(l1ls_instance* I) {
    if (!I) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(I->device);
    (void)hipDeviceSynchronize();
    I->arena.release();
    (void)hipSetDevice(cur);
    delete I;
}
