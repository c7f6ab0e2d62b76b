// Batched FISTA: many instances of problem (1) advanced together (section
// 8.1 FISTA on each), FP32 bulk over each instance's stored CSR/CSC.
//
// Every resident instance ("slot") keeps its own device state: iteration
// count k, momentum t_k and beta, gap and converged flag, so instances that
// joined at different times run side by side.  One launch runs the transpose
// pass of all slots and one the residual pass, over a table of 64-row
// (64-column) tiles tagged with their slot; a per-slot tail kernel evaluates
// the gap on that slot's check iterations and advances its momentum state.
// Tiles never mix slots and each slot's partial sums are reduced in a fixed
// order, so a slot's iterates and its convergence test are bit-for-bit the
// same alone and in any mix of other slots.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

using namespace l1ls;

struct BInst {  // static per slot
    const int32_t* csr_ptr;
    const int32_t* csr_col;
    const float* csr_val;
    const int32_t* csc_ptr;
    const int32_t* csc_row;
    const float* csc_val;
    const float* b;
    float* x[2];
    float* rx;
    float* ry;
    int64_t m, n;
    double tau, L, tol;
    int64_t max_iter;                             // <= 0: no cap
    int32_t t1_begin, t1_end, t2_begin, t2_end;  // this slot's tiles in the tables
    int32_t check_every, pad;
};

struct BState {  // dynamic per slot
    int64_t k;          // iterations done
    double t;           // t_{k+1}
    double beta_prev;   // beta_k, used by the next transpose pass
    double P, D, gap;
    int64_t conv_iter;  // -1 until the gap test passes
    int32_t active, done, nonfinite, init_pending;
    int32_t stale;      // tile tables were rebuilt: previous-parity partials are void
    int32_t pad;
};

struct BTile {
    int32_t slot;
    int32_t first;  // first row (column) of the 64-tile
};

namespace {

// t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2 with the same operation order as the
// single-instance driver ((4 t) t), so both produce the same beta bits.
__device__ __forceinline__ double next_t_dev(double t) {
    return __ddiv_rn(__dadd_rn(1.0, __dsqrt_rn(__dadd_rn(1.0, __dmul_rn(__dmul_rn(4.0, t), t)))), 2.0);
}

__device__ __forceinline__ bool slot_runs(const BState& st, int mode) {
    return mode == 1 ? (st.active && st.init_pending) : (st.active && !st.done && !st.init_pending);
}

// Transpose pass of iteration k+1 of every running slot.
__global__ __launch_bounds__(L1LS_BLOCK) void kb_transpose(const BTile* __restrict__ tiles, int32_t ntiles,
                                                           const BInst* __restrict__ bi,
                                                           const BState* __restrict__ bs,
                                                           double* __restrict__ k2part) {
    __shared__ float lds[L1LS_BLOCK / L1LS_WAVE][kTile * kMaxNnz];
    const int lane = threadIdx.x % L1LS_WAVE, wid = threadIdx.x / L1LS_WAVE;
    const int32_t tile = (int32_t)blockIdx.x * (L1LS_BLOCK / L1LS_WAVE) + wid;
    bool run = false;
    BTile tl{0, 0};
    if (tile < ntiles) {
        tl = tiles[tile];
        run = slot_runs(bs[tl.slot], 0);
    }
    const BInst& I = bi[tl.slot];
    const BState& S = bs[tl.slot];
    const int64_t j = (int64_t)tl.first + lane;
    const bool live = run && j < I.n;
    const int64_t k = S.k;
    const float* xc = I.x[k & 1];
    float* xp = I.x[(k + 1) & 1];
    int32_t pb = 0, pe = 0;
    float xcur = 0.f, xprev = 0.f;
    if (live) {
        pb = I.csc_ptr[j];
        pe = I.csc_ptr[j + 1];
        xcur = xc[j];
        xprev = xp[j];
    }
    int32_t beg = 0, end = 0;
    if (run) {
        const int lastlane = (tl.first + kTile <= I.n) ? kTile - 1 : (int)(I.n - tl.first - 1);
        beg = __builtin_amdgcn_readfirstlane(__shfl(pb, 0, L1LS_WAVE));
        end = __builtin_amdgcn_readfirstlane(__shfl(pe, lastlane, L1LS_WAVE));
        tile_products<float, 16>(I.csc_row, I.csc_val, I.ry, beg, end - beg, lds[wid], lane);
    }
    __syncthreads();
    if (!run) return;
    double v[2] = {0.0, 0.0};  // sum |x|, max |g|
    if (live) {
        float acc = 0.f;
        for (int32_t q = pb - beg; q < pe - beg; ++q) acc += lds[wid][q];
        const float beta = (float)S.beta_prev;
        const float y = xcur + beta * (xcur - xprev);
        const float xn = soft_threshold<float>(y - acc / (float)I.L, (float)(I.tau / I.L));
        xp[j] = xn;
        v[0] = fabs((double)xn);
        v[1] = fabs((double)acc);
    }
    v[0] = wave_sum(v[0]);
    v[1] = wave_max(v[1]);
    if (lane == 0) {
        k2part[2 * tile + 0] = v[1];
        k2part[2 * tile + 1] = v[0];
    }
}

// Residual pass of iteration k+1 (mode 0) or the first pass r = A x_0 - b
// of slots just admitted (mode 1); partial sums go to parity slot (k+1) & 1
// (0 for mode 1).
__global__ __launch_bounds__(L1LS_BLOCK) void kb_residual(const BTile* __restrict__ tiles, int32_t ntiles,
                                                          const BInst* __restrict__ bi,
                                                          const BState* __restrict__ bs,
                                                          double* __restrict__ k1part, int32_t ntiles_total,
                                                          int mode) {
    __shared__ float lds[L1LS_BLOCK / L1LS_WAVE][kTile * kMaxNnz];
    const int lane = threadIdx.x % L1LS_WAVE, wid = threadIdx.x / L1LS_WAVE;
    const int32_t tile = (int32_t)blockIdx.x * (L1LS_BLOCK / L1LS_WAVE) + wid;
    bool run = false;
    BTile tl{0, 0};
    if (tile < ntiles) {
        tl = tiles[tile];
        run = slot_runs(bs[tl.slot], mode);
    }
    const BInst& I = bi[tl.slot];
    const BState& S = bs[tl.slot];
    const int64_t i = (int64_t)tl.first + lane;
    const bool live = run && i < I.m;
    const int64_t k1 = (mode == 1) ? 0 : S.k + 1;
    const float* x = I.x[k1 & 1];
    int32_t pb = 0, pe = 0;
    float b = 0.f, rprev = 0.f;
    if (live) {
        pb = I.csr_ptr[i];
        pe = I.csr_ptr[i + 1];
        b = I.b[i];
        if (mode == 0) rprev = I.rx[i];
    }
    int32_t beg = 0, end = 0;
    if (run) {
        const int lastlane = (tl.first + kTile <= I.m) ? kTile - 1 : (int)(I.m - tl.first - 1);
        beg = __builtin_amdgcn_readfirstlane(__shfl(pb, 0, L1LS_WAVE));
        end = __builtin_amdgcn_readfirstlane(__shfl(pe, lastlane, L1LS_WAVE));
        tile_products<float, 10>(I.csr_col, I.csr_val, x, beg, end - beg, lds[wid], lane);
    }
    __syncthreads();
    if (!run) return;
    // beta_{k+1} = (t_{k+1} - 1) / t_{k+2}
    const float beta = (mode == 1) ? 0.f : (float)((S.t - 1.0) / next_t_dev(S.t));
    double v[3] = {0.0, 0.0, 0.0};
    if (live) {
        float acc = 0.f;
        for (int32_t q = pb - beg; q < pe - beg; ++q) acc += lds[wid][q];
        const float r = acc - b;
        const float yv = (mode == 1) ? r : (1.f + beta) * r - beta * rprev;
        I.rx[i] = r;
        I.ry[i] = yv;
        v[0] = (double)r * (double)r;
        v[1] = (double)yv * (double)yv;
        v[2] = (double)b * (double)yv;
    }
    for (int q = 0; q < 3; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0) {
        double* p = k1part + (size_t)(k1 & 1) * 3 * ntiles_total + 3 * (size_t)tile;
        p[0] = v[0];
        p[1] = v[1];
        p[2] = v[2];
    }
}

// One workgroup per slot: gap test on check iterations, then advance t, beta, k.
__global__ __launch_bounds__(256) void kb_tail(const BInst* __restrict__ bi, BState* __restrict__ bs,
                                               const double* __restrict__ k1part, const double* __restrict__ k2part,
                                               int32_t ntiles_total, int mode) {
    const int slot = blockIdx.x;
    BState& S = bs[slot];
    const BInst& I = bi[slot];
    if (mode == 1) {
        if (threadIdx.x == 0 && S.active && S.init_pending) S.init_pending = 0;
        return;
    }
    if (!slot_runs(S, 0)) return;
    const int64_t kn = S.k + 1;
    const bool eval = (kn % I.check_every == 0) && !S.stale;
    __syncthreads();  // every thread has read S before thread 0 writes it
    bool stop = false;
    if (eval) {
        const double* cur = k1part + (size_t)(kn & 1) * 3 * ntiles_total;
        const double* prev = k1part + (size_t)((kn - 1) & 1) * 3 * ntiles_total;
        double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // rr, ryy, bry, l1 | ginf
        for (int t = I.t1_begin + threadIdx.x; t < I.t1_end; t += blockDim.x) {
            v[0] += cur[3 * t];
            v[1] += prev[3 * t + 1];
            v[2] += prev[3 * t + 2];
        }
        for (int t = I.t2_begin + threadIdx.x; t < I.t2_end; t += blockDim.x) {
            v[3] += k2part[2 * t + 1];
            v[4] = fmax(v[4], k2part[2 * t]);
        }
        block_reduce_stats<5, 4>(v);
        if (threadIdx.x == 0) {
            const double P = I.tau * v[3] + 0.5 * v[0];
            const double theta = (v[4] <= I.tau) ? 1.0 : I.tau / v[4];
            const double D = -0.5 * theta * theta * v[1] - theta * v[2];
            const double gap = (P - D) / fabs(P);
            S.P = P;
            S.D = D;
            S.gap = gap;
            const bool finite = (P == P) && (D == D) && (P - P == 0.0) && (D - D == 0.0);
            if (!finite) {
                S.nonfinite = 1;
                stop = true;
            } else if (I.tol > 0.0 && gap <= I.tol) {
                S.conv_iter = kn;
                stop = true;
            }
        }
    }
    if (threadIdx.x == 0) {
        S.stale = 0;
        if (I.max_iter > 0 && kn >= I.max_iter) stop = true;  // iteration cap: done, not converged
        if (stop) {
            S.done = 1;
            S.k = kn;
        } else {
            const double tn = next_t_dev(S.t);
            S.beta_prev = (S.t - 1.0) / tn;
            S.t = tn;
            S.k = kn;
        }
    }
}

// After the tile tables change, the previous-parity partial sums of running
// slots sit at stale positions: skip their next gap evaluation.
__global__ void kb_mark_stale(BState* __restrict__ bs, int32_t capacity) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < capacity && bs[s].active && !bs[s].init_pending) bs[s].stale = 1;
}

__global__ void kb_zero(float* __restrict__ a, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) a[i] = 0.f;
}

__global__ void kb_to_f64_perm(const float* __restrict__ x, double* __restrict__ out, const int32_t* __restrict__ pos,
                               int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) out[j] = (double)x[pos ? pos[j] : j];
}

inline dim3 g1d(int64_t N) { return dim3((unsigned)std::max<int64_t>(1, (N + L1LS_BLOCK - 1) / L1LS_BLOCK)); }

}  // namespace

struct l1ls_batch {
    int32_t capacity = 0;
    size_t budget = 0, used = 0;
    hipStream_t stream = nullptr;
    l1ls_solve_opts o;
    std::vector<const l1ls_instance*> inst;   // per slot (nullptr: free)
    std::vector<BInst> hinst;
    std::vector<size_t> footprint;
    std::vector<std::vector<float*>> bufs;    // per-slot device buffers
    BInst* dinst = nullptr;
    BState* dstate = nullptr;
    BTile* dt1 = nullptr;
    BTile* dt2 = nullptr;
    int32_t cap1 = 0, cap2 = 0, nt1 = 0, nt2 = 0;
    double* k1part = nullptr;
    double* k2part = nullptr;
    bool tables_dirty = false, init_pending = false;
    DevArena arena;
};

namespace {

size_t slot_footprint(const l1ls_instance* I) {
    // iterate buffers of the slot (the instance's own arrays are counted by
    // the caller's admission policy through l1ls_instance_footprint)
    return (size_t)(2 * I->n + 2 * I->m) * sizeof(float);
}

l1ls_status rebuild_tables(l1ls_batch* B) {
    std::vector<BTile> t1, t2;
    for (int s = 0; s < B->capacity; ++s) {
        BInst& hi = B->hinst[s];
        if (!B->inst[s]) continue;
        hi.t1_begin = (int32_t)t1.size();
        for (int64_t r = 0; r < hi.m; r += kTile) t1.push_back(BTile{s, (int32_t)r});
        hi.t1_end = (int32_t)t1.size();
        hi.t2_begin = (int32_t)t2.size();
        for (int64_t c = 0; c < hi.n; c += kTile) t2.push_back(BTile{s, (int32_t)c});
        hi.t2_end = (int32_t)t2.size();
    }
    if ((int32_t)t1.size() > B->cap1 || (int32_t)t2.size() > B->cap2) {
        // grow the tile tables and partial arrays (old ones stay in the arena)
        B->cap1 = std::max<int32_t>((int32_t)t1.size(), 2 * B->cap1);
        B->cap2 = std::max<int32_t>((int32_t)t2.size(), 2 * B->cap2);
        L1LS_TRY(B->arena.alloc(&B->dt1, B->cap1));
        L1LS_TRY(B->arena.alloc(&B->dt2, B->cap2));
        L1LS_TRY(B->arena.alloc(&B->k1part, (size_t)2 * 3 * B->cap1));
        L1LS_TRY(B->arena.alloc(&B->k2part, (size_t)2 * B->cap2));
    }
    B->nt1 = (int32_t)t1.size();
    B->nt2 = (int32_t)t2.size();
    if (!t1.empty())
        HIP_TRY(hipMemcpyAsync(B->dt1, t1.data(), t1.size() * sizeof(BTile), hipMemcpyHostToDevice, B->stream));
    if (!t2.empty())
        HIP_TRY(hipMemcpyAsync(B->dt2, t2.data(), t2.size() * sizeof(BTile), hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipMemcpyAsync(B->dinst, B->hinst.data(), B->capacity * sizeof(BInst), hipMemcpyHostToDevice, B->stream));
    hipLaunchKernelGGL(kb_mark_stale, dim3((B->capacity + 255) / 256), dim3(256), 0, B->stream, B->dstate,
                       B->capacity);
    HIP_TRY(hipGetLastError());
    // the copies read host vectors that go out of scope: wait for them
    HIP_TRY(hipStreamSynchronize(B->stream));
    B->tables_dirty = false;
    return L1LS_OK;
}

l1ls_status run_init(l1ls_batch* B) {
    if (B->nt1 == 0) return L1LS_OK;
    const int g1 = (B->nt1 + 3) / 4;
    hipLaunchKernelGGL(kb_residual, dim3(g1), dim3(L1LS_BLOCK), 0, B->stream, B->dt1, B->nt1, B->dinst, B->dstate,
                       B->k1part, B->cap1, 1);
    hipLaunchKernelGGL(kb_tail, dim3(B->capacity), dim3(256), 0, B->stream, B->dinst, B->dstate, B->k1part,
                       B->k2part, B->cap1, 1);
    HIP_TRY(hipGetLastError());
    B->init_pending = false;
    return L1LS_OK;
}

}  // namespace

extern "C" l1ls_status l1ls_batch_create(int32_t capacity, size_t hbm_budget_bytes, const l1ls_solve_opts* opts,
                                         l1ls_batch** out) {
    if (!out || !opts || capacity < 1 || capacity > 65535) return L1LS_E_ARG;
    *out = nullptr;
    if (opts->precision != L1LS_F32 || opts->op != L1LS_OP_STORED) return L1LS_E_UNSUPPORTED;
    if (opts->check_every < 1 || !(opts->rel_gap_tol >= 0.0)) return L1LS_E_ARG;
    l1ls_batch* B = new l1ls_batch();
    B->capacity = capacity;
    B->budget = hbm_budget_bytes;
    B->stream = (hipStream_t)opts->stream;
    B->o = *opts;
    B->inst.assign(capacity, nullptr);
    B->hinst.assign(capacity, BInst{});
    B->footprint.assign(capacity, 0);
    B->bufs.assign(capacity, {});
    auto fail = [&](l1ls_status s) {
        B->arena.release();
        delete B;
        return s;
    };
    l1ls_status st;
    if ((st = B->arena.alloc(&B->dinst, capacity)) != L1LS_OK) return fail(st);
    if ((st = B->arena.alloc(&B->dstate, capacity)) != L1LS_OK) return fail(st);
    if (hipMemsetAsync(B->dstate, 0, capacity * sizeof(BState), B->stream) != hipSuccess) return fail(L1LS_E_HIP);
    if (hipMemsetAsync(B->dinst, 0, capacity * sizeof(BInst), B->stream) != hipSuccess) return fail(L1LS_E_HIP);
    if (hipStreamSynchronize(B->stream) != hipSuccess) return fail(L1LS_E_HIP);
    *out = B;
    return L1LS_OK;
}

extern "C" size_t l1ls_instance_footprint(const l1ls_instance* I) {
    if (!I) return 0;
    // stored FP32 CSR + CSC, FP64 copies if kept, vectors and tables, plus the
    // batch slot's iterate buffers
    size_t b = 0;
    if (I->csr_v32) b += (size_t)I->nnz * 16 + (size_t)(I->m + I->n + 2) * 4;
    if (I->csr_v64) b += (size_t)I->nnz * 16;
    b += (size_t)(I->m + I->n) * 48;
    return b + slot_footprint(I);
}

extern "C" l1ls_status l1ls_batch_add_ex(l1ls_batch* B, const l1ls_instance* I, double tau, double rel_gap_tol,
                                         int64_t max_iter, int32_t* slot_out) {
    if (!B || !I || !slot_out) return L1LS_E_ARG;
    if (rel_gap_tol != rel_gap_tol) return L1LS_E_ARG;
    *slot_out = -1;
    if (!I->csr_v32 || !I->csc_v32) return L1LS_E_UNSUPPORTED;
    if (!(tau > 0.0) || !is_finite(tau)) tau = I->tau;
    int slot = -1;
    for (int s = 0; s < B->capacity; ++s)
        if (!B->inst[s]) {
            slot = s;
            break;
        }
    if (slot < 0) return L1LS_E_STATE;  // no free slot
    const size_t fp = l1ls_instance_footprint(I);
    if (B->budget && B->used + fp > B->budget) return L1LS_E_NOMEM;
    std::vector<float*> bufs(4, nullptr);
    for (int q = 0; q < 4; ++q) {
        const int64_t N = (q < 2) ? I->n : I->m;
        void* p = nullptr;
        if (hipMalloc(&p, N * sizeof(float)) != hipSuccess) {
            for (float* f : bufs)
                if (f) (void)hipFree(f);
            return L1LS_E_NOMEM;
        }
        bufs[q] = (float*)p;
        hipLaunchKernelGGL(kb_zero, g1d(N), dim3(L1LS_BLOCK), 0, B->stream, bufs[q], N);
    }
    BInst& h = B->hinst[slot];
    h.csr_ptr = I->csr_ptr;
    h.csr_col = I->csr_col;
    h.csr_val = I->csr_v32;
    h.csc_ptr = I->csc_ptr;
    h.csc_row = I->csc_row;
    h.csc_val = I->csc_v32;
    h.b = I->b32_op;
    h.x[0] = bufs[0];
    h.x[1] = bufs[1];
    h.rx = bufs[2];
    h.ry = bufs[3];
    h.m = I->m;
    h.n = I->n;
    h.tau = tau;
    h.L = I->L;
    h.tol = rel_gap_tol >= 0.0 ? rel_gap_tol : B->o.rel_gap_tol;
    h.max_iter = max_iter > 0 ? max_iter : 0;
    h.check_every = B->o.check_every;
    B->inst[slot] = I;
    B->bufs[slot] = bufs;
    B->footprint[slot] = fp;
    B->used += fp;
    BState s0;
    std::memset(&s0, 0, sizeof(s0));
    s0.t = 1.0;
    s0.conv_iter = -1;
    s0.active = 1;
    s0.init_pending = 1;
    HIP_TRY(hipMemcpyAsync(B->dstate + slot, &s0, sizeof(s0), hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    B->tables_dirty = true;
    B->init_pending = true;
    *slot_out = slot;
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_batch_add(l1ls_batch* B, const l1ls_instance* I, double tau, int32_t* slot_out) {
    return l1ls_batch_add_ex(B, I, tau, -1.0, 0, slot_out);
}

extern "C" l1ls_status l1ls_batch_iterate(l1ls_batch* B, int64_t iters) {
    if (!B || iters < 0) return L1LS_E_ARG;
    if (B->tables_dirty) L1LS_TRY(rebuild_tables(B));
    if (B->init_pending) L1LS_TRY(run_init(B));
    if (B->nt1 == 0) return L1LS_OK;
    const int g1 = (B->nt1 + 3) / 4, g2 = (B->nt2 + 3) / 4;
    for (int64_t q = 0; q < iters; ++q) {
        hipLaunchKernelGGL(kb_transpose, dim3(g2), dim3(L1LS_BLOCK), 0, B->stream, B->dt2, B->nt2, B->dinst,
                           B->dstate, B->k2part);
        hipLaunchKernelGGL(kb_residual, dim3(g1), dim3(L1LS_BLOCK), 0, B->stream, B->dt1, B->nt1, B->dinst,
                           B->dstate, B->k1part, B->cap1, 0);
        hipLaunchKernelGGL(kb_tail, dim3(B->capacity), dim3(256), 0, B->stream, B->dinst, B->dstate, B->k1part,
                           B->k2part, B->cap1, 0);
    }
    HIP_TRY(hipGetLastError());
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_batch_poll(l1ls_batch* B, l1ls_report* reports, int32_t* active_out) {
    if (!B || !reports) return L1LS_E_ARG;
    std::vector<BState> st(B->capacity);
    HIP_TRY(hipMemcpyAsync(st.data(), B->dstate, B->capacity * sizeof(BState), hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    int32_t act = 0;
    for (int s = 0; s < B->capacity; ++s) {
        l1ls_report& r = reports[s];
        std::memset(&r, 0, sizeof(r));
        if (!B->inst[s]) {
            r.iterations = -1;
            continue;
        }
        r.iterations = (st[s].conv_iter >= 0) ? st[s].conv_iter : st[s].k;
        r.primal = st[s].P;
        r.dual = st[s].D;
        r.rel_gap = st[s].gap;
        r.converged = st[s].conv_iter >= 0 ? 1 : (st[s].nonfinite ? -1 : 0);
        r.rel_err = -1.0;
        if (!st[s].done) ++act;
    }
    if (active_out) *active_out = act;
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_batch_get_x(l1ls_batch* B, int32_t slot, double* x_out) {
    if (!B || !x_out || slot < 0 || slot >= B->capacity || !B->inst[slot]) return L1LS_E_ARG;
    BState st;
    HIP_TRY(hipMemcpyAsync(&st, B->dstate + slot, sizeof(st), hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    const l1ls_instance* I = B->inst[slot];
    hipLaunchKernelGGL(kb_to_f64_perm, g1d(I->n), dim3(L1LS_BLOCK), 0, B->stream, B->hinst[slot].x[st.k & 1], x_out,
                       I->op_col_pos, I->n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(B->stream));
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_batch_remove(l1ls_batch* B, int32_t slot) {
    if (!B || slot < 0 || slot >= B->capacity || !B->inst[slot]) return L1LS_E_ARG;
    HIP_TRY(hipStreamSynchronize(B->stream));
    BState s0;
    std::memset(&s0, 0, sizeof(s0));
    s0.conv_iter = -1;
    HIP_TRY(hipMemcpyAsync(B->dstate + slot, &s0, sizeof(s0), hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    for (float* f : B->bufs[slot]) (void)hipFree(f);
    B->bufs[slot].clear();
    B->used -= B->footprint[slot];
    B->footprint[slot] = 0;
    B->inst[slot] = nullptr;
    B->hinst[slot] = BInst{};
    B->tables_dirty = true;
    return L1LS_OK;
}

extern "C" void l1ls_batch_destroy(l1ls_batch* B) {
    if (!B) return;
    (void)hipStreamSynchronize(B->stream);
    for (auto& v : B->bufs)
        for (float* f : v) (void)hipFree(f);
    B->arena.release();
    delete B;
}

extern "C" l1ls_status l1ls_solve_fista_batched(const l1ls_instance* const* insts, const double* taus, int32_t count,
                                                const l1ls_solve_opts* opts, double* const* x_outs,
                                                l1ls_report* reports) {
    if (!insts || !opts || !x_outs || !reports || count < 1) return L1LS_E_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    l1ls_batch* B = nullptr;
    L1LS_TRY(l1ls_batch_create(count, 0, opts, &B));
    l1ls_status st = L1LS_OK;
    std::vector<int32_t> slot(count, -1);
    for (int q = 0; q < count && st == L1LS_OK; ++q) st = l1ls_batch_add(B, insts[q], taus ? taus[q] : 0.0, &slot[q]);
    std::vector<l1ls_report> rep(count);
    const int64_t chunk = (int64_t)opts->check_every * 4;
    int64_t done_iters = 0;
    while (st == L1LS_OK && done_iters < opts->max_iter) {
        const int64_t step = std::min<int64_t>(chunk, opts->max_iter - done_iters);
        if ((st = l1ls_batch_iterate(B, step)) != L1LS_OK) break;
        done_iters += step;
        int32_t act = 0;
        if ((st = l1ls_batch_poll(B, rep.data(), &act)) != L1LS_OK) break;
        if (act == 0) break;
    }
    if (st == L1LS_OK) st = l1ls_batch_poll(B, rep.data(), nullptr);
    bool all = true;
    for (int q = 0; q < count && st == L1LS_OK; ++q) {
        st = l1ls_batch_get_x(B, slot[q], x_outs[q]);
        reports[q] = rep[slot[q]];
        all = all && reports[q].converged == 1;
    }
    l1ls_batch_destroy(B);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int q = 0; q < count; ++q) reports[q].seconds = secs;
    if (st != L1LS_OK) return st;
    return all ? L1LS_OK : L1LS_NOT_CONVERGED;
}
