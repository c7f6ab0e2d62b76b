// Windowed gathers for the stored FP32 passes (the products of section 8.1's
// FISTA over the stored CSR/CSC of A).
//
// The CSR pass gathers x at the columns of its rows: in stage order a row's
// columns form a few runs of four at random places (the Sigma embedding
// links two independent bijections), so once x no longer fits the caches
// each run costs a cache line.  The windowed form groups the targets (rows
// of the CSR pass, columns of the CSC pass) in windows of consecutive
// positions and keeps, per window, one copy of each source element the
// window reads, in a bucketed vector u ordered by window, then by source
// chunk (2^14 consecutive sources).  A bucketing pass copies the sources
// into u chunk by chunk (the chunk staged in LDS, each window's run of the
// chunk written with consecutive stores); the pass itself then gathers
// u[idx'] with idx' the slot of its (window, source) pair, and a window's
// segment of u (about 1 MB) stays in one XCD's L2 while the window's
// workgroups run (they are placed on one XCD, kernels.hpp).  The values
// gathered are the same, so the results are bitwise those of the plain
// passes.
//
// Tables (built once per instance, L1LS_STORE_WINDOWS): for every window,
// in one launch per window, the first entry naming a source claims it
// (atomic exchange of a per-source mark) and takes the next slot of its
// (window, chunk) run; a second launch per window writes the slot of every
// entry.  The order within a run depends on the claims' timing, not the
// results.
#include <algorithm>
#include <cstdint>

#include "common.hpp"

l1ls_status exclusive_scan_i32(const int32_t* counts, int32_t* offsets, int64_t n, hipStream_t stream,
                               DevArena& tmp);

namespace {

constexpr int kSwCs = 14;           // sources per chunk: 2^14 (64 KB of FP32 staging)
constexpr int kSwThreads = 1024;
constexpr int64_t kSwSlotsPerWindow = (int64_t)1 << 18;  // about 1 MB of FP32 per window segment

inline dim3 g1d(int64_t N) { return dim3((unsigned)std::max<int64_t>(1, (N + L1LS_BLOCK - 1) / L1LS_BLOCK)); }

// Window w = targets [t0, t1): entries claim their source (mark) the first
// time the window meets it.  phase 0: count claims per (window, chunk);
// phase 1: take a slot (cursor), record it (slotof) and its source offset.
__global__ void k_sw_claim(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx, int64_t t0, int64_t t1,
                           int32_t tag, int64_t w, int64_t nc, int32_t* __restrict__ mark, int32_t* __restrict__ cnt,
                           int32_t* __restrict__ cursor, int32_t* __restrict__ slotof, uint16_t* __restrict__ src) {
    const int64_t t = t0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= t1) return;
    for (int32_t e = ptr[t]; e < ptr[t + 1]; ++e) {
        const int32_t j = idx[e];
        if (atomicExch(&mark[j], tag) == tag) continue;  // claimed already in this window
        const int64_t run = w * nc + (j >> kSwCs);
        if (!cursor) {
            atomicAdd(&cnt[run], 1);
        } else {
            const int32_t slot = atomicAdd(&cursor[run], 1);
            slotof[j] = slot;
            src[slot] = (uint16_t)(j & ((1 << kSwCs) - 1));
        }
    }
}

// The slot of every entry of window [t0, t1).
__global__ void k_sw_fill(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx, int64_t t0, int64_t t1,
                          const int32_t* __restrict__ slotof, int32_t* __restrict__ out) {
    const int64_t t = t0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= t1) return;
    for (int32_t e = ptr[t]; e < ptr[t + 1]; ++e) out[e] = slotof[idx[e]];
}

// The runs in chunk-major order for the bucketing pass: run (w, c) spans
// slots [start[c nT + w], end[c nT + w]).
__global__ void k_sw_runs(const int32_t* __restrict__ base, int64_t nT, int64_t nc, int32_t* __restrict__ start,
                          int32_t* __restrict__ end) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nT * nc) return;
    const int64_t w = q / nc, c = q - w * nc;
    start[c * nT + w] = base[q];
    end[c * nT + w] = base[q + 1];
}

__global__ void k_sw_fill_i32(int32_t* __restrict__ a, int32_t v, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) a[i] = v;
}

}  // namespace

// Tables of side k (0: CSR over m rows gathering from n sources, 1: CSC over
// n columns gathering from m sources).
l1ls_status build_windows_side(l1ls_instance* I, int k, hipStream_t s) {
    const int64_t T = k == 0 ? I->m : I->n;  // targets
    const int64_t S = k == 0 ? I->n : I->m;  // sources
    const int32_t* ptr = k == 0 ? I->csr_ptr : I->csc_ptr;
    const int32_t* idx = k == 0 ? I->csr_col : I->csc_row;
    // windows of a power-of-two number of targets, about kSwSlotsPerWindow
    // slots each (every entry at most one slot)
    int64_t per = 1;
    while (per < T && (I->nnz / std::max<int64_t>(T, 1)) * per * 2 <= kSwSlotsPerWindow * 4) per *= 2;
    const int64_t nT = (T + per - 1) / per;
    const int64_t nc = (S + ((int64_t)1 << kSwCs) - 1) >> kSwCs;
    if (nT * nc + 1 >= ((int64_t)1 << 31)) return L1LS_E_UNSUPPORTED;
    DevArena tmp;
    tmp.al = I->arena.al;
    auto fail = [&](l1ls_status st) {
        (void)hipStreamSynchronize(s);
        tmp.release();
        return st;
    };
    int32_t *mark = nullptr, *cnt = nullptr, *base = nullptr, *cursor = nullptr, *slotof = nullptr;
    int32_t *rs = nullptr, *re = nullptr;
    l1ls_status st;
    if ((st = tmp.alloc(&mark, S)) != L1LS_OK) return fail(st);
    if ((st = tmp.alloc(&slotof, S)) != L1LS_OK) return fail(st);
    if ((st = tmp.alloc(&cnt, nT * nc + 1)) != L1LS_OK) return fail(st);
    if ((st = tmp.alloc(&cursor, nT * nc + 1)) != L1LS_OK) return fail(st);
    if ((st = tmp.alloc(&base, nT * nc + 1)) != L1LS_OK) return fail(st);
    if ((st = I->arena.alloc(&rs, nT * nc)) != L1LS_OK) return fail(st);
    if ((st = I->arena.alloc(&re, nT * nc)) != L1LS_OK) return fail(st);
    hipLaunchKernelGGL(k_sw_fill_i32, g1d(S), dim3(L1LS_BLOCK), 0, s, mark, -1, S);
    hipLaunchKernelGGL(k_sw_fill_i32, g1d(nT * nc + 1), dim3(L1LS_BLOCK), 0, s, cnt, 0, nT * nc + 1);
    for (int64_t w = 0; w < nT; ++w) {
        const int64_t t0 = w * per, t1 = std::min(T, t0 + per);
        hipLaunchKernelGGL(k_sw_claim, g1d(t1 - t0), dim3(L1LS_BLOCK), 0, s, ptr, idx, t0, t1, (int32_t)w, w, nc,
                           mark, cnt, (int32_t*)nullptr, (int32_t*)nullptr, (uint16_t*)nullptr);
    }
    if ((st = exclusive_scan_i32(cnt, base, nT * nc, s, tmp)) != L1LS_OK) return fail(st);
    int32_t total = 0;
    if (hipMemcpyAsync(&total, base + nT * nc, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(L1LS_E_HIP);
    // the passes gather with 32-bit byte offsets
    if ((int64_t)total * (int64_t)sizeof(float) >= ((int64_t)1 << 32)) return fail(L1LS_E_UNSUPPORTED);
    uint16_t* src = nullptr;
    int32_t* out = nullptr;
    if ((st = I->arena.alloc(&src, std::max<int64_t>(total, 1))) != L1LS_OK) return fail(st);
    if ((st = I->arena.alloc(&out, I->nnz)) != L1LS_OK) return fail(st);
    if (hipMemcpyAsync(cursor, base, (nT * nc + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(L1LS_E_HIP);
    hipLaunchKernelGGL(k_sw_fill_i32, g1d(S), dim3(L1LS_BLOCK), 0, s, mark, -1, S);
    for (int64_t w = 0; w < nT; ++w) {
        const int64_t t0 = w * per, t1 = std::min(T, t0 + per);
        hipLaunchKernelGGL(k_sw_claim, g1d(t1 - t0), dim3(L1LS_BLOCK), 0, s, ptr, idx, t0, t1, (int32_t)w, w, nc,
                           mark, cnt, cursor, slotof, src);
        hipLaunchKernelGGL(k_sw_fill, g1d(t1 - t0), dim3(L1LS_BLOCK), 0, s, ptr, idx, t0, t1,
                           (const int32_t*)slotof, out);
    }
    hipLaunchKernelGGL(k_sw_runs, g1d(nT * nc), dim3(L1LS_BLOCK), 0, s, (const int32_t*)base, nT, nc, rs, re);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return fail(L1LS_E_HIP);
    tmp.release();
    I->sw_idx[k] = out;
    I->sw_src[k] = src;
    I->sw_start[k] = rs;
    I->sw_end[k] = re;
    I->sw_slots[k] = total;
    I->sw_nT[k] = nT;
    I->sw_nc[k] = nc;
    I->sw_cs[k] = kSwCs;
    return L1LS_OK;
}

l1ls_status build_stored_windows(l1ls_instance* I, hipStream_t s) {
    if (!I->csr_ptr || !I->csc_ptr) return L1LS_E_UNSUPPORTED;
    L1LS_TRY(build_windows_side(I, 0, s));
    L1LS_TRY(build_windows_side(I, 1, s));
    return L1LS_OK;
}

namespace {

// u = the bucketed copy of src (N sources) for side k: one workgroup per
// chunk stages the chunk in LDS, then its waves copy the chunk's run of each
// window (window-major runs, consecutive slots).
template <typename T>
__global__ __launch_bounds__(kSwThreads) void k_sw_scatter(const T* __restrict__ src, int64_t N,
                                                           const int32_t* __restrict__ start,
                                                           const int32_t* __restrict__ end, int64_t nT,
                                                           const uint16_t* __restrict__ off, T* __restrict__ u,
                                                           const int32_t* __restrict__ done) {
    __shared__ T st[1 << kSwCs];
    if (done && *done) return;  // the solver's converged flag (launch-uniform)
    const int64_t c = blockIdx.x;
    const int64_t c0 = c << kSwCs;
    const int cnt = (int)std::min<int64_t>((int64_t)1 << kSwCs, N - c0);
    for (int j = threadIdx.x; j < cnt; j += kSwThreads) st[j] = src[c0 + j];
    __syncthreads();
    const int lane = threadIdx.x % L1LS_WAVE, wave = threadIdx.x / L1LS_WAVE;
    const int32_t* sc = start + c * nT;
    const int32_t* ec = end + c * nT;
    for (int64_t w = wave; w < nT; w += kSwThreads / L1LS_WAVE) {
        const int32_t b = sc[w], e = ec[w];
        for (int32_t q = b + lane; q < e; q += L1LS_WAVE) u[q] = st[off[q]];
    }
}

}  // namespace

// u_k = bucketed copy of src for side k (0: x, n sources; 1: r_y, m sources).
void stored_window_scatter(const l1ls_instance* I, int k, const float* src, float* u, const int32_t* done,
                           hipStream_t s) {
    const int64_t N = k == 0 ? I->n : I->m;
    hipLaunchKernelGGL((k_sw_scatter<float>), dim3((unsigned)I->sw_nc[k]), dim3(kSwThreads), 0, s, src, N,
                       (const int32_t*)I->sw_start[k], (const int32_t*)I->sw_end[k], I->sw_nT[k],
                       (const uint16_t*)I->sw_src[k], u, done);
}
