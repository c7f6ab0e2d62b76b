// Windowed gathers for the stored FP32 passes (the products of section 8.1's
// FISTA over the stored CSR/CSC of A).
//
// The CSR pass gathers x at the columns of its rows: in stage order a row's
// columns form a few runs of four consecutive positions at random places
// (the Sigma embedding links two independent bijections), shared by the few
// neighbouring rows of one rotation group.  Once x no longer fits the caches
// each run costs a whole cache line of HBM traffic for 16 useful bytes.  The
// windowed form groups the targets (rows of the CSR pass, columns of the CSC
// pass) in windows of consecutive positions and keeps, per window, one copy
// of each unit the window reads, a unit being 4 consecutive source elements
// starting where a row's run starts.  The copies form a bucketed vector u
// ordered by source chunk (2^14 consecutive sources), then by window.  A
// bucketing pass fills u chunk by chunk (the chunk staged in LDS, the units
// of the chunk written with consecutive 16-byte stores); the pass itself
// then gathers u at 4 unit + offset, whole lines of u that stay in one XCD's
// L2 while the window's workgroups run (they are placed on one XCD,
// kernels.hpp).  The values gathered are the same, so the results are
// bitwise those of the plain passes.
//
// Tables (built once per instance, L1LS_STORE_WINDOWS): every entry's offset
// from the start of its unit (a row's entries in order; a unit starts at an
// entry that does not follow the previous one within 4 positions); then, for
// every window, in one launch per window, the first entry that starts a unit
// claims it (atomic exchange of a per-source mark) and takes the next unit of
// its (chunk, window) run; a second launch per window writes the position in
// u of every entry.  The order within a run depends on the claims' timing,
// not the results.
#include <algorithm>
#include <cstdint>

#include "common.hpp"

l1ls_status exclusive_scan_i32(const int32_t* counts, int32_t* offsets, int64_t n, hipStream_t stream,
                               DevArena& tmp);

namespace {

constexpr int kSwCs = 14;          // sources per chunk: 2^14 (64 KB of FP32 staging)
constexpr int kSwUnit = 4;         // sources per unit
constexpr int kSwThreads = 1024;
constexpr int64_t kSwEntriesPerWindow = (int64_t)1 << 20;  // about 1 MB of u per window at two stages

inline dim3 g1d(int64_t N) { return dim3((unsigned)std::max<int64_t>(1, (N + L1LS_BLOCK - 1) / L1LS_BLOCK)); }

// delta[e] = idx[e] - (start of e's unit): a target's entries in order, a
// new unit wherever an entry does not lie above the previous one within
// kSwUnit positions of the current unit's start.
__global__ void k_sw_delta(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx, int64_t T,
                           uint8_t* __restrict__ delta) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    int32_t s = 0, prev = 0;
    const int32_t b = ptr[t], e1 = ptr[t + 1];
    for (int32_t e = b; e < e1; ++e) {
        const int32_t j = idx[e];
        if (e == b || j <= prev || j - s >= kSwUnit) s = j;
        delta[e] = (uint8_t)(j - s);
        prev = j;
    }
}

// Window w = targets [t0, t1): entries that start a unit claim it (mark) the
// first time the window meets it.  phase 0 (cursor null): count claims per
// (chunk, window); phase 1: take a unit (cursor), record it (unitof) and the
// offset of its start in its chunk (src).
__global__ void k_sw_claim(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                           const uint8_t* __restrict__ delta, int64_t t0, int64_t t1, int32_t tag, int64_t w,
                           int64_t nT, int32_t* __restrict__ mark, int32_t* __restrict__ cnt,
                           int32_t* __restrict__ cursor, int32_t* __restrict__ unitof, uint16_t* __restrict__ src) {
    const int64_t t = t0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= t1) return;
    for (int32_t e = ptr[t]; e < ptr[t + 1]; ++e) {
        if (delta[e] != 0) continue;
        const int32_t j = idx[e];
        if (atomicExch(&mark[j], tag) == tag) continue;  // claimed already in this window
        const int64_t run = (int64_t)(j >> kSwCs) * nT + w;
        if (!cursor) {
            atomicAdd(&cnt[run], 1);
        } else {
            const int32_t q = atomicAdd(&cursor[run], 1);
            unitof[j] = q;
            src[q] = (uint16_t)(j & ((1 << kSwCs) - 1));
        }
    }
}

// The position in u of every entry of window [t0, t1).
__global__ void k_sw_fill(const int32_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                          const uint8_t* __restrict__ delta, int64_t t0, int64_t t1,
                          const int32_t* __restrict__ unitof, int32_t* __restrict__ out) {
    const int64_t t = t0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= t1) return;
    for (int32_t e = ptr[t]; e < ptr[t + 1]; ++e) {
        const int32_t d = delta[e];
        out[e] = kSwUnit * unitof[idx[e] - d] + d;
    }
}

// cb[c] = first unit of chunk c (c = 0..nc).
__global__ void k_sw_chunks(const int32_t* __restrict__ base, int64_t nT, int64_t nc, int32_t* __restrict__ cb) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c <= nc) cb[c] = base[c * nT];
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
    // windows of a power-of-two number of targets, about kSwEntriesPerWindow
    // entries each
    int64_t per = 1;
    while (per < T && (I->nnz / std::max<int64_t>(T, 1)) * per * 2 <= kSwEntriesPerWindow) per *= 2;
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
    int32_t *mark = nullptr, *cnt = nullptr, *base = nullptr, *cursor = nullptr, *unitof = nullptr, *cb = nullptr;
    uint8_t* delta = nullptr;
    l1ls_status st;
    if ((st = tmp.alloc(&delta, std::max<int64_t>(I->nnz, 1))) != L1LS_OK) return fail(st);
    if ((st = tmp.alloc(&mark, S)) != L1LS_OK) return fail(st);
    if ((st = tmp.alloc(&unitof, S)) != L1LS_OK) return fail(st);
    if ((st = tmp.alloc(&cnt, nT * nc + 1)) != L1LS_OK) return fail(st);
    if ((st = tmp.alloc(&cursor, nT * nc + 1)) != L1LS_OK) return fail(st);
    if ((st = tmp.alloc(&base, nT * nc + 1)) != L1LS_OK) return fail(st);
    if ((st = I->arena.alloc(&cb, nc + 1)) != L1LS_OK) return fail(st);
    hipLaunchKernelGGL(k_sw_delta, g1d(T), dim3(L1LS_BLOCK), 0, s, ptr, idx, T, delta);
    hipLaunchKernelGGL(k_sw_fill_i32, g1d(S), dim3(L1LS_BLOCK), 0, s, mark, -1, S);
    hipLaunchKernelGGL(k_sw_fill_i32, g1d(nT * nc + 1), dim3(L1LS_BLOCK), 0, s, cnt, 0, nT * nc + 1);
    for (int64_t w = 0; w < nT; ++w) {
        const int64_t t0 = w * per, t1 = std::min(T, t0 + per);
        hipLaunchKernelGGL(k_sw_claim, g1d(t1 - t0), dim3(L1LS_BLOCK), 0, s, ptr, idx, (const uint8_t*)delta, t0, t1,
                           (int32_t)w, w, nT, mark, cnt, (int32_t*)nullptr, (int32_t*)nullptr, (uint16_t*)nullptr);
    }
    if ((st = exclusive_scan_i32(cnt, base, nT * nc, s, tmp)) != L1LS_OK) return fail(st);
    int32_t units = 0;
    if (hipMemcpyAsync(&units, base + nT * nc, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(L1LS_E_HIP);
    // the passes gather with 32-bit byte offsets into u (4 floats per unit)
    if ((int64_t)units * kSwUnit * (int64_t)sizeof(float) >= ((int64_t)1 << 32)) return fail(L1LS_E_UNSUPPORTED);
    uint16_t* src = nullptr;
    int32_t* out = nullptr;
    // one spare entry: the bucketing pass reads offsets two at a time
    if ((st = I->arena.alloc(&src, (int64_t)units + 2)) != L1LS_OK) return fail(st);
    if ((st = I->arena.alloc(&out, std::max<int64_t>(I->nnz, 1))) != L1LS_OK) return fail(st);
    if (hipMemcpyAsync(cursor, base, (nT * nc + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(L1LS_E_HIP);
    hipLaunchKernelGGL(k_sw_fill_i32, g1d(S), dim3(L1LS_BLOCK), 0, s, mark, -1, S);
    for (int64_t w = 0; w < nT; ++w) {
        const int64_t t0 = w * per, t1 = std::min(T, t0 + per);
        hipLaunchKernelGGL(k_sw_claim, g1d(t1 - t0), dim3(L1LS_BLOCK), 0, s, ptr, idx, (const uint8_t*)delta, t0, t1,
                           (int32_t)w, w, nT, mark, cnt, cursor, unitof, src);
        hipLaunchKernelGGL(k_sw_fill, g1d(t1 - t0), dim3(L1LS_BLOCK), 0, s, ptr, idx, (const uint8_t*)delta, t0, t1,
                           (const int32_t*)unitof, out);
    }
    hipLaunchKernelGGL(k_sw_chunks, g1d(nc + 1), dim3(L1LS_BLOCK), 0, s, (const int32_t*)base, nT, nc, cb);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return fail(L1LS_E_HIP);
    tmp.release();
    I->sw_idx[k] = out;
    I->sw_src[k] = src;
    I->sw_cb[k] = cb;
    I->sw_slots[k] = (int64_t)units * kSwUnit;
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

// u = the bucketed copy of src (N sources) for one side: one workgroup per
// chunk stages the chunk and the 3 sources after it in LDS (zero past N),
// then writes the chunk's units (consecutive in u) as 16-byte stores, two
// consecutive units per thread and step.  Every global load a thread needs
// for the stores (the staging float4s and its first kSwPairs pairs of unit
// offsets, read as 32-bit words) is issued before the barrier, so the stores
// never wait behind a load: the vector memory counter counts loads and stores
// in one order, and a load issued after a store would make the store's
// completion part of the wait.
constexpr int kSwPairs = 9;  // 2 x 9 x 1024 units per chunk before the tail loop (about 16K expected)

__global__ __launch_bounds__(kSwThreads) void k_sw_scatter(const float* __restrict__ src, int64_t N,
                                                           const int32_t* __restrict__ cb,
                                                           const uint16_t* __restrict__ off, float4* __restrict__ u,
                                                           const int32_t* __restrict__ done) {
    constexpr int kC = 1 << kSwCs;
    __shared__ __align__(16) float st[kC + 8];
    if (done && *done) return;  // the solver's converged flag (launch-uniform)
    const int tid = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x << kSwCs;
    const int cnt = (int)std::min<int64_t>(kC, N - c0);
    const int32_t q0 = cb[blockIdx.x], q1 = cb[blockIdx.x + 1];
    // unit pairs (2p, 2p + 1) for p from q0 / 2: 32-bit loads of two offsets
    const int32_t p0 = q0 >> 1;
    const uint32_t* off2 = reinterpret_cast<const uint32_t*>(off);
    const int32_t p1 = (q1 + 1) >> 1;
    uint32_t o[kSwPairs];
#pragma unroll
    for (int k = 0; k < kSwPairs; ++k) {
        const int32_t p = p0 + tid + k * kSwThreads;
        o[k] = p < p1 ? __builtin_nontemporal_load(off2 + p) : 0u;
    }
    const float* s0 = src + c0;
    const int n4 = cnt >> 2;
    if ((reinterpret_cast<uintptr_t>(s0) & 15) == 0) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        f4 a[kC / 4 / kSwThreads];
#pragma unroll
        for (int k = 0; k < kC / 4 / kSwThreads; ++k) {
            const int i = tid + k * kSwThreads;
            a[k] = i < n4 ? __builtin_nontemporal_load(reinterpret_cast<const f4*>(s0) + i) : f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int k = 0; k < kC / 4 / kSwThreads; ++k) {
            const int i = tid + k * kSwThreads;
            if (i < n4) reinterpret_cast<f4*>(st)[i] = a[k];
        }
    } else {
        for (int j = tid; j < 4 * n4; j += kSwThreads) st[j] = s0[j];
    }
    // the last cnt mod 4 sources and the 3 after the chunk (zero past N)
    if (tid < 8) {
        const int j = 4 * n4 + tid;
        if (j < cnt + kSwUnit - 1) st[j] = c0 + j < N ? s0[j] : 0.0f;
    }
    __syncthreads();
    auto put = [&](int32_t p, uint32_t w) {
        const int32_t q = 2 * p;
        if (q >= q0 && q < q1) {
            const int a = (int)(w & 0xffffu);
            u[q] = make_float4(st[a], st[a + 1], st[a + 2], st[a + 3]);
        }
        if (q + 1 >= q0 && q + 1 < q1) {
            const int a = (int)(w >> 16);
            u[q + 1] = make_float4(st[a], st[a + 1], st[a + 2], st[a + 3]);
        }
    };
#pragma unroll
    for (int k = 0; k < kSwPairs; ++k) put(p0 + tid + k * kSwThreads, o[k]);
    for (int32_t p = p0 + tid + kSwPairs * kSwThreads; p < p1; p += kSwThreads) put(p, off2[p]);
}

}  // namespace

// u_k = bucketed copy of src for side k (0: x, n sources; 1: r_y, m sources).
void stored_window_scatter(const l1ls_instance* I, int k, const float* src, float* u, const int32_t* done,
                           hipStream_t s) {
    const int64_t N = k == 0 ? I->n : I->m;
    hipLaunchKernelGGL(k_sw_scatter, dim3((unsigned)I->sw_nc[k]), dim3(kSwThreads), 0, s, src, N,
                       (const int32_t*)I->sw_cb[k], (const uint16_t*)I->sw_src[k], reinterpret_cast<float4*>(u),
                       done);
}
