// Shared internals of the l1ls HIP library: status helpers, the instance
// object, wave64 reductions and the deterministic FP64 block reduction.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/l1ls.h"

#define L1LS_MAX_ROUNDS 2
#define L1LS_WAVE 64
#define L1LS_BLOCK 256

// Return L1LS_E_HIP from the enclosing function when a HIP call fails.
#define HIP_TRY(expr)                                                        \
    do {                                                                     \
        hipError_t _e = (expr);                                              \
        if (_e != hipSuccess) {                                              \
            if (std::getenv("L1LS_DEBUG"))                                   \
                std::fprintf(stderr, "l1ls: %s failed: %s (%s:%d)\n", #expr, \
                             hipGetErrorString(_e), __FILE__, __LINE__);     \
            return _e == hipErrorOutOfMemory ? L1LS_E_NOMEM : L1LS_E_HIP;    \
        }                                                                    \
    } while (0)

#define L1LS_TRY(expr)                        \
    do {                                      \
        l1ls_status _s = (expr);              \
        if (_s != L1LS_OK) return _s;         \
    } while (0)

// A source of device memory.  The default (no DevAlloc) is hipMalloc /
// hipFree; hipFree waits for all work queued on the device, so a caller that
// allocates and frees while other streams run (the serving loop) supplies a
// caching allocator instead.  free() is only called once nothing in flight
// uses the block.
struct DevAlloc {
    virtual ~DevAlloc() = default;
    virtual l1ls_status alloc(void** p, size_t bytes) = 0;
    virtual void free(void* p, size_t bytes) = 0;
};

// Device memory of the process-wide source (alloc.hip): the allocator
// installed with l1ls_set_allocator, else hipMalloc / hipFree.  lib_free
// returns a block to whichever source made it.
// synced: the caller has waited for the device since the block's last use.
l1ls_status lib_alloc(void** p, size_t bytes);
void lib_free(void* p, size_t bytes, bool synced = false);

inline l1ls_status dev_alloc(DevAlloc* al, void** p, size_t bytes) {
    *p = nullptr;
    if (al) return al->alloc(p, bytes);
    return lib_alloc(p, bytes);
}

inline void dev_free(DevAlloc* al, void* p, size_t bytes, bool synced = false) {
    if (!p) return;
    if (al)
        al->free(p, bytes);
    else
        lib_free(p, bytes, synced);
}

// Device allocation list owned by one object; freed in reverse order.
struct DevArena {
    std::vector<std::pair<void*, size_t>> ptrs;
    DevAlloc* al = nullptr;
    template <typename T>
    l1ls_status alloc(T** p, size_t count) {
        *p = nullptr;
        if (count == 0) count = 1;
        void* q = nullptr;
        L1LS_TRY(dev_alloc(al, &q, count * sizeof(T)));
        ptrs.push_back({q, count * sizeof(T)});
        *p = static_cast<T*>(q);
        return L1LS_OK;
    }
    void release() {
        // one wait for the device covers every block (hipFree would wait once per block)
        if (!al && !ptrs.empty()) (void)hipDeviceSynchronize();
        for (size_t i = ptrs.size(); i-- > 0;) dev_free(al, ptrs[i].first, ptrs[i].second, true);
        ptrs.clear();
    }
    // Free one block of the list (nothing queued may still use it; nullptr:
    // nothing to do).
    void free_one(void* p) {
        if (!p) return;
        for (size_t i = 0; i < ptrs.size(); ++i)
            if (ptrs[i].first == p) {
                dev_free(al, p, ptrs[i].second);
                ptrs.erase(ptrs.begin() + (long)i);
                return;
            }
    }
};

// Pair tables of one side: bijection pi (position -> index), its inverse,
// and per stage the (c, s) of each of the N/2 rotations (FP64, interleaved).
struct SideTables {
    int64_t N = 0;
    int32_t* perm = nullptr;
    int32_t* pinv = nullptr;
    double* cs[L1LS_MAX_ROUNDS] = {nullptr, nullptr};
};

struct l1ls_instance {
    int64_t m = 0, n = 0, s = 0, nnz = 0;
    int32_t rounds = 1;
    bool igen2 = false;           // m < n: Procedure IGen2 (igen2.hip); stored operator only
    uint32_t storage = 0;
    int32_t layout = 0;
    double kappa = 1, tau = 1, L = 1, fstar = 0;
    uint64_t seed = 0;
    int device = 0;
    SideTables side[2];           // [0] = n side (G), [1] = m side (Q)
    double* sigma = nullptr;      // n
    double* xstar = nullptr;      // n
    double* g = nullptr;          // n
    double* e = nullptr;          // m
    double* b = nullptr;          // m
    float* b32 = nullptr;         // m
    int32_t* support = nullptr;   // s
    double* colnorm2 = nullptr;   // n, diag(A^T A), original order
    // Operator order (the order of the stored CSR/CSC): b and diag(A^T A)
    // permuted; op_col_of[p] / op_row_of[p] give the original index at
    // position p, op_col_pos / op_row_pos the inverse (nullptr: identity).
    double* b_op = nullptr;
    float* b32_op = nullptr;
    double* colnorm2_op = nullptr;
    const int32_t* op_col_of = nullptr;
    const int32_t* op_col_pos = nullptr;
    const int32_t* op_row_of = nullptr;
    const int32_t* op_row_pos = nullptr;
    // Matrix-free operator in stage order (see mf.hip): Sigma links
    // m-position i and n-position mf_emb[i] (or none, -1); mf_inv[a] = rank,
    // among the active m-positions, of the one linked to n-position a;
    // mf_cbase[g] = active m-positions before workgroup g's first (2 g B);
    // mf_sig* = sigma at m-positions (0 if none).
    int32_t* mf_emb = nullptr;
    int32_t* mf_inv = nullptr;
    int32_t* mf_cbase = nullptr;
    // Windowed gathers of the matrix-free passes (mfw_ws = 0: off); [0] is
    // the m side's gather of w, [1] the n side's gather of the compact v.
    // Target positions are grouped in windows of 2^mfw_ws, sources in chunks
    // of 2^mfw_cs[k]; mfw_ib[k][t] = slot of the bucketed copy u that target
    // position t reads (-1 where the position is inactive); mfw_lx[k][src] =
    // place of source element src in its chunk's staging order (offset by
    // the chunk's start), and mfw_wslot[k][j] = slot of u that staging place j
    // is written to.
    int mfw_ws = 0;
    int mfw_cs[2] = {0, 0};
    int32_t* mfw_ib[2] = {nullptr, nullptr};
    int32_t* mfw_lx[2] = {nullptr, nullptr};
    int32_t* mfw_wslot[2] = {nullptr, nullptr};
    double* mf_sig64 = nullptr;
    float* mf_sig32 = nullptr;
    double* mf_sign64 = nullptr;  // sigma at n-positions
    float* mf_sign32 = nullptr;
    double* mf_b64 = nullptr;     // b in m-stage order
    float* mf_b32 = nullptr;
    float* mf_cs32[2][L1LS_MAX_ROUNDS] = {{nullptr, nullptr}, {nullptr, nullptr}};
    int32_t* csr_ptr = nullptr;   // m+1
    int32_t* csr_col = nullptr;
    double* csr_v64 = nullptr;
    float* csr_v32 = nullptr;
    int32_t* csc_ptr = nullptr;   // n+1
    int32_t* csc_row = nullptr;
    double* csc_v64 = nullptr;
    float* csc_v32 = nullptr;
    // Blocked operator (two stages, stage order; see blocks.hip): row runs
    // (pointer, start, 4 FP32 values each) and exactly four runs per column
    // (slot h of column a at h * n + a).  Starts index the extended layout.
    int32_t* blk_rptr = nullptr;  // m+1
    int32_t* blk_rstart = nullptr;
    float* blk_rval = nullptr;    // 4 per run
    int32_t* blk_cstart = nullptr;  // 4n
    float* blk_cval = nullptr;    // 4 per run
    int64_t blk_nruns = 0;
    // Windowed gathers of the stored FP32 passes (L1LS_STORE_WINDOWS; see
    // window.hip).  [0]: the CSR pass's gather of x (row windows), [1]: the
    // CSC pass's gather of r_y (column windows).  The bucketed copy u_k is
    // made of units of 4 consecutive source elements; sw_idx[k] replaces the
    // CSR column (CSC row) indices by positions in u_k (4 unit + offset);
    // sw_src[k][unit] = offset of the unit's first source in its chunk of
    // 2^sw_cs sources; the units of chunk c are [sw_cb[k][c], sw_cb[k][c+1])
    // (chunk-major, then window).  sw_slots[k] = 4 units (floats of u_k).
    int32_t* sw_idx[2] = {nullptr, nullptr};
    uint16_t* sw_src[2] = {nullptr, nullptr};
    int32_t* sw_cb[2] = {nullptr, nullptr};
    int64_t sw_slots[2] = {0, 0};
    int64_t sw_nT[2] = {0, 0};
    int64_t sw_nc[2] = {0, 0};
    int sw_cs[2] = {0, 0};
    DevArena arena;
};

// ---------------------------------------------------------------------------
// wave64 / block reductions
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = L1LS_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, L1LS_WAVE);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = L1LS_WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, L1LS_WAVE));
    return v;
}

// Sum over a segment of W consecutive lanes (W a power of two <= 64); every
// lane of the segment ends with the segment total.
template <int W, typename T>
__device__ __forceinline__ T segment_sum(T v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}

// Deterministic block reduction of NS FP64 statistics: stats with index in
// [0, NSUM) are summed, the rest take the maximum.  The result is valid in
// thread 0.  Fixed order: butterfly inside each wave, then waves in order.
template <int NS, int NSUM>
__device__ __forceinline__ void block_reduce_stats(double (&v)[NS]) {
    __shared__ double red[1024 / L1LS_WAVE][NS];
    const int lane = threadIdx.x % L1LS_WAVE;
    const int wid = threadIdx.x / L1LS_WAVE;
#pragma unroll
    for (int i = 0; i < NS; ++i) v[i] = (i < NSUM) ? wave_sum(v[i]) : wave_max(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NS; ++i) red[wid][i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            double a = red[0][i];
            for (int w = 1; w < (int)(blockDim.x / L1LS_WAVE); ++w)
                a = (i < NSUM) ? a + red[w][i] : fmax(a, red[w][i]);
            v[i] = a;
        }
    }
    __syncthreads();
}

inline int grid_for(int64_t work_items, int items_per_block, int cap) {
    int64_t g = (work_items + items_per_block - 1) / items_per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// out[p] = in[of[p]] (gather into operator order; of == nullptr: copy).
template <typename Tout, typename Tin>
__global__ void k_gather_perm(const Tin* __restrict__ in, Tout* __restrict__ out, const int32_t* __restrict__ of,
                              int64_t N) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    out[p] = (Tout)in[of ? of[p] : p];
}

inline dim3 grid_1d(int64_t N) {
    return dim3((unsigned)((N + L1LS_BLOCK - 1) / L1LS_BLOCK > 0 ? (N + L1LS_BLOCK - 1) / L1LS_BLOCK : 1));
}

// Exclusive prefix sum of int32 counts into int32 offsets (n+1 outputs).
l1ls_status exclusive_scan_i32(const int32_t* counts, int32_t* offsets, int64_t n,
                               hipStream_t stream, DevArena& tmp);

// Host-side checks of pointer validity for the ABI.
inline bool is_finite(double v) { return v == v && v - v == 0.0; }
