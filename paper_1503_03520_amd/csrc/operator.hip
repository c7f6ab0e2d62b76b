// Matrix-free products with A = Q Sigma G^T (section 4, Algorithms MvPA and
// MvPAt): the Givens stages are applied from the pair tables, Sigma scales
// and embeds R^n into R^m (or truncates and scales back), no A is stored.
#include "common.hpp"
#include "stages.hpp"

using namespace l1ls;

template <typename T>
l1ls_status apply_side(const SideTables& tab, int rounds, bool transpose, T* v, T* scratch, hipStream_t stream);

namespace {

// z_k = sigma_k w_k for k < n, 0 for n <= k < m
template <typename T>
__global__ void k_sigma_embed(const T* __restrict__ w, T* __restrict__ z, const double* __restrict__ sigma,
                              int64_t n, int64_t m) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    z[k] = (k < n) ? (T)sigma[k] * w[k] : T(0);
}

// w_k = sigma_k z_k for k < n
template <typename T>
__global__ void k_sigma_truncate(const T* __restrict__ z, T* __restrict__ w, const double* __restrict__ sigma,
                                 int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    w[k] = (T)sigma[k] * z[k];
}

inline dim3 g1d(int64_t N) { return dim3((unsigned)std::max<int64_t>(1, (N + L1LS_BLOCK - 1) / L1LS_BLOCK)); }

}  // namespace

template <typename T>
l1ls_status apply_matrix_free(const l1ls_instance* I, int trans, const T* in, T* out, hipStream_t s) {
    DevArena tmp;
    T *wn = nullptr, *wn2 = nullptr, *zm = nullptr, *zm2 = nullptr;
    auto done = [&](l1ls_status st) {
        tmp.release();
        return st;
    };
    l1ls_status st;
    if ((st = tmp.alloc(&wn, I->n)) != L1LS_OK) return done(st);
    if ((st = tmp.alloc(&wn2, I->n)) != L1LS_OK) return done(st);
    if ((st = tmp.alloc(&zm, I->m)) != L1LS_OK) return done(st);
    if ((st = tmp.alloc(&zm2, I->m)) != L1LS_OK) return done(st);
    if (trans == 0) {
        // MvPA: G^T (its factors in order), Sigma, then Q (last factor first)
        if (hipMemcpyAsync(wn, in, I->n * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
            return done(L1LS_E_HIP);
        if ((st = apply_side<T>(I->side[0], I->rounds, true, wn, wn2, s)) != L1LS_OK) return done(st);
        hipLaunchKernelGGL(k_sigma_embed<T>, g1d(I->m), dim3(L1LS_BLOCK), 0, s, wn, zm, I->sigma, I->n, I->m);
        if ((st = apply_side<T>(I->side[1], I->rounds, false, zm, zm2, s)) != L1LS_OK) return done(st);
        if (hipMemcpyAsync(out, zm, I->m * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
            return done(L1LS_E_HIP);
    } else {
        // MvPAt: Q^T, Sigma^T, then G
        if (hipMemcpyAsync(zm, in, I->m * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
            return done(L1LS_E_HIP);
        if ((st = apply_side<T>(I->side[1], I->rounds, true, zm, zm2, s)) != L1LS_OK) return done(st);
        hipLaunchKernelGGL(k_sigma_truncate<T>, g1d(I->n), dim3(L1LS_BLOCK), 0, s, zm, wn, I->sigma, I->n);
        if ((st = apply_side<T>(I->side[0], I->rounds, false, wn, wn2, s)) != L1LS_OK) return done(st);
        if (hipMemcpyAsync(out, wn, I->n * sizeof(T), hipMemcpyDeviceToDevice, s) != hipSuccess)
            return done(L1LS_E_HIP);
    }
    if (hipGetLastError() != hipSuccess) return done(L1LS_E_HIP);
    if (hipStreamSynchronize(s) != hipSuccess) return done(L1LS_E_HIP);
    return done(L1LS_OK);
}
template l1ls_status apply_matrix_free<double>(const l1ls_instance*, int, const double*, double*, hipStream_t);
template l1ls_status apply_matrix_free<float>(const l1ls_instance*, int, const float*, float*, hipStream_t);
