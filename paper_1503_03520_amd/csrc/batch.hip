// Batched FISTA: many instances of problem (1) advanced together (section
// 8.1 FISTA on each), FP32 bulk over each instance's stored CSR/CSC.
//
// The batch counts global iterations G.  A slot ("resident instance")
// records the G at which it was admitted, so its own iteration number is
// k = G - admit and instances that joined at different times run side by
// side.  The momentum coefficients beta_k depend on k alone: a host-built
// table (same arithmetic as the single-instance driver) serves every slot.
// One launch runs the transpose pass of all slots and one the residual pass,
// over a table of 64-row (64-column) tiles tagged with their slot; the gap
// kernel runs on the iterations where some slot reaches a check iteration.
// Tiles never mix slots, each slot keeps its partial sums in its own buffer
// (indexed by its own tile number) and reduces them in a fixed order, so a
// slot's iterates and its convergence test are bit-for-bit the same alone
// and in any mix of other slots.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "tune.hpp"

using namespace l1ls;

struct BInst {  // static per slot (device copy refreshed on add/remove)
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
    double* part1;  // [2 parities][nt1][3]: ||r_x||^2, ||r_y||^2, b^T r_y per row tile
    double* part2;  // [nt2][2]: max |A^T r_y|, sum |x| per column tile
    int64_t m, n;
    int64_t admit;     // G when x_0 was set: the slot's iteration k = G - admit
    int64_t max_iter;  // <= 0: no cap
    double tau, L, tol;
    int32_t nt1, nt2;
    int32_t check_every, active;
    int32_t admit_mod;  // admit mod check_every
    int32_t persist;    // 1: the slot's iterations run in kb_persist (one workgroup), not in the shared passes
};

struct BState {  // written by the gap kernel only
    double P, D, gap;
    int64_t stop_iter;  // iteration at which the slot stopped (done = 1)
    int32_t done, converged, nonfinite, pad;
};

// A workgroup's share of one slot's pass: `steps` rounds of 4 consecutive
// 64-row (64-column) tiles from row (column) `first`; wave w takes tile
// 4 s + w of round s.  The number of rounds per task is the tile schedule,
// chosen per slot size by the autotuner (more rounds amortise the slot
// lookups of a workgroup; fewer keep small slots spread over more CUs).
struct BTask {
    int32_t slot;
    int32_t first;
    int32_t steps;
    int32_t pad;
};

namespace {

// A slot's iteration number in global iteration G, and whether it runs then.
__device__ __forceinline__ bool slot_live(const BInst& I, const BState& S, int64_t G, int64_t* kn) {
    *kn = G - I.admit;
    return I.active && !S.done && *kn >= 1 && (I.max_iter <= 0 || *kn <= I.max_iter);
}

// k mod check_every for the slot, from gmod = G mod check_every (32-bit).
__device__ __forceinline__ int slot_phase(const BInst& I, int gmod) {
    const int r = gmod - I.admit_mod;
    return r < 0 ? r + I.check_every : r;
}

// One 64-column tile of the transpose pass (pointers as restrict parameters:
// inlined, the compiler keeps their no-alias scopes).
__device__ __forceinline__ void transpose_tile(const int32_t* __restrict__ ptr, const int32_t* __restrict__ row,
                                               const float* __restrict__ val, const float* __restrict__ ry,
                                               const float* __restrict__ xc, float* __restrict__ xp,
                                               double* __restrict__ part2, int64_t n, int64_t first, float beta,
                                               float Lf, float thr, bool stats, bool more, float* lds, int lane) {
    const bool run = first < n;  // wave-uniform
    const int64_t j = first + lane;
    const bool live = run && j < n;
    int32_t pb = 0, pe = 0;
    float xcur = 0.f, xprev = 0.f;
    if (live) {
        pb = ptr[j];
        pe = ptr[j + 1];
        xcur = __builtin_nontemporal_load(xc + j);
        xprev = __builtin_nontemporal_load(xp + j);
    }
    if (run) {
        const int lastlane = (first + kTile <= n) ? kTile - 1 : (int)(n - first - 1);
        const int32_t beg = __builtin_amdgcn_readfirstlane(__shfl(pb, 0, L1LS_WAVE));
        const int32_t end = __builtin_amdgcn_readfirstlane(__shfl(pe, lastlane, L1LS_WAVE));
        tile_products<float, 16>(row, val, ry, beg, end - beg, lds, lane);
        pb -= beg;
        pe -= beg;
    }
    __syncthreads();
    double v[2] = {0.0, 0.0};  // sum |x_k|, max |g|
    if (live) {
        float acc = 0.f;
        for (int32_t q = pb; q < pe; ++q) acc += lds[q];
        const float y = xcur + beta * (xcur - xprev);
        const float xn = soft_threshold<float>(y - acc / Lf, thr);
        st_stream(xp + j, xn);
        v[0] = fabs((double)xn);
        v[1] = fabs((double)acc);
    }
    if (run && stats) {
        v[0] = wave_sum(v[0]);
        v[1] = wave_max(v[1]);
        if (lane == 0) {
            double* p = part2 + 2 * (size_t)(first / kTile);
            p[0] = v[1];
            p[1] = v[0];
        }
    }
    if (more) __syncthreads();  // the wave's LDS slice is rewritten by the next round
}

// Transpose pass of global iteration G: x_k = soft(y_k - A^T r_y,k / L), with
// y_k = x_{k-1} + beta_{k-1} (x_{k-1} - x_{k-2}).  ONE: every task is a single
// round (no loop; the register budget of the single-instance kernel).  The
// occupancy hints are the largest without register spills.
template <bool ONE>
__global__ __launch_bounds__(L1LS_BLOCK, ONE ? 7 : 5) void kb_transpose(const BTask* __restrict__ tasks,
                                                           const BInst* __restrict__ bi,
                                                           const BState* __restrict__ bs,
                                                           const float* __restrict__ btab,
                                                           const int64_t* __restrict__ dG, int64_t Gh, int ce) {
    __shared__ float lds[L1LS_BLOCK / L1LS_WAVE][kTile * kMaxNnz];
    const int lane = threadIdx.x % L1LS_WAVE;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / L1LS_WAVE);
    // the iteration this launch runs: from the device count (graph replays)
    // or from the argument (launched one by one)
    const int64_t G = (dG ? *dG : Gh) + 1;
    const int gmod = (int)(G % ce);
    const BTask tk = tasks[blockIdx.x];
    const BInst& I = bi[tk.slot];
    int64_t kn = 0;
    if (!slot_live(I, bs[tk.slot], G, &kn)) return;  // block-uniform
    const bool stats = slot_phase(I, gmod) == 0;    // a gap test reads this pass
    const float beta = btab[kn - 1];
    const float Lf = (float)I.L, thr = (float)(I.tau / I.L);
    const int steps = ONE ? 1 : tk.steps;
    for (int st = 0; st < steps; ++st)
        transpose_tile(I.csc_ptr, I.csc_row, I.csc_val, I.ry, I.x[(kn - 1) & 1], I.x[kn & 1], I.part2, I.n,
                       (int64_t)tk.first + (int64_t)(4 * st + wid) * kTile, beta, Lf, thr, stats, st + 1 < steps,
                       lds[wid], lane);
}

// One 64-row tile of the residual pass (mode 1: first pass, no momentum).
__device__ __forceinline__ void residual_tile(const int32_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                              const float* __restrict__ val, const float* __restrict__ x,
                                              const float* __restrict__ bvec, float* __restrict__ rx,
                                              float* __restrict__ ry, double* __restrict__ part1, int64_t m,
                                              int64_t first, float beta, int mode, bool stats, bool more, float* lds,
                                              int lane) {
    const bool run = first < m;  // wave-uniform
    const int64_t i = first + lane;
    const bool live = run && i < m;
    int32_t pb = 0, pe = 0;
    float b = 0.f, rprev = 0.f;
    if (live) {
        pb = ptr[i];
        pe = ptr[i + 1];
        b = __builtin_nontemporal_load(bvec + i);
        if (mode == 0) rprev = __builtin_nontemporal_load(rx + i);
    }
    if (run) {
        const int lastlane = (first + kTile <= m) ? kTile - 1 : (int)(m - first - 1);
        const int32_t beg = __builtin_amdgcn_readfirstlane(__shfl(pb, 0, L1LS_WAVE));
        const int32_t end = __builtin_amdgcn_readfirstlane(__shfl(pe, lastlane, L1LS_WAVE));
        tile_products<float, 10>(col, val, x, beg, end - beg, lds, lane);
        pb -= beg;
        pe -= beg;
    }
    __syncthreads();
    double v[3] = {0.0, 0.0, 0.0};
    if (live) {
        float acc = 0.f;
        for (int32_t q = pb; q < pe; ++q) acc += lds[q];
        const float r = acc - b;
        const float yv = (mode == 1) ? r : (1.f + beta) * r - beta * rprev;
        st_stream(rx + i, r);
        st_stream(ry + i, yv);
        v[0] = (double)r * (double)r;
        v[1] = (double)yv * (double)yv;
        v[2] = (double)b * (double)yv;
    }
    if (run && stats) {
        for (int q = 0; q < 3; ++q) v[q] = wave_sum(v[q]);
        if (lane == 0) {
            double* p = part1 + (size_t)(first / kTile) * 3;
            p[0] = v[0];
            p[1] = v[1];
            p[2] = v[2];
        }
    }
    if (more) __syncthreads();  // the wave's LDS slice is rewritten by the next round
}

// Residual pass of global iteration G (mode 0): r_x,k = A x_k - b and
// r_y,k+1 = (1 + beta_k) r_x,k - beta_k r_x,k-1; or, for the slots admitted
// at G (mode 1), the first pass r_x,0 = r_y,1 = A x_0 - b.  Partial sums go
// to parity k & 1 of the slot's buffer (0 for mode 1).
template <bool ONE>
__global__ __launch_bounds__(L1LS_BLOCK, 8) void kb_residual(const BTask* __restrict__ tasks,
                                                          const BInst* __restrict__ bi,
                                                          const BState* __restrict__ bs,
                                                          const float* __restrict__ btab,
                                                          const int64_t* __restrict__ dG, int64_t Gh, int ce,
                                                          int mode) {
    __shared__ float lds[L1LS_BLOCK / L1LS_WAVE][kTile * kMaxNnz];
    const int lane = threadIdx.x % L1LS_WAVE;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / L1LS_WAVE);
    // as kb_transpose; mode 1 (first passes) runs at the current count G
    const int64_t G = (dG ? *dG : Gh) + (mode == 1 ? 0 : 1);
    const int gmod = (int)(G % ce);
    const BTask tk = tasks[blockIdx.x];
    const BInst& I = bi[tk.slot];
    int64_t kn = 0;
    if (mode == 1) {
        if (!(I.active && I.admit == G)) return;  // block-uniform
    } else if (!slot_live(I, bs[tk.slot], G, &kn)) {
        return;
    }
    // a gap test at k reads ||r_x,k|| from this pass, and the r_y terms of
    // the pass of k - 1 (the point whose gradient the transpose pass of k used)
    bool stats = true;
    if (mode == 0) {
        const int ph = slot_phase(I, gmod);
        stats = (ph == 0 || ph == I.check_every - 1);
    }
    const float beta = (mode == 1) ? 0.f : btab[kn];
    double* part1 = I.part1 + (size_t)(kn & 1) * I.nt1 * 3;
    const int steps = ONE ? 1 : tk.steps;
    for (int st = 0; st < steps; ++st)
        residual_tile(I.csr_ptr, I.csr_col, I.csr_val, I.x[kn & 1], I.b, I.rx, I.ry, part1, I.m,
                      (int64_t)tk.first + (int64_t)(4 * st + wid) * kTile, beta, mode, stats, st + 1 < steps,
                      lds[wid], lane);
}

// The duality gap of one slot at its iteration kn (a check iteration), by a
// workgroup of 1024 threads: the terms of k_gap, from the slot's own partials
// in tile order.
__device__ __forceinline__ void slot_gap(const BInst& I, BState& S, int64_t kn) {
    const double* cur = I.part1 + (size_t)(kn & 1) * 3 * I.nt1;
    const double* prev = I.part1 + (size_t)((kn - 1) & 1) * 3 * I.nt1;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // rr, ryy, bry, l1 | ginf
    for (int t = threadIdx.x; t < I.nt1; t += blockDim.x) {
        v[0] += cur[3 * t];
        v[1] += prev[3 * t + 1];
        v[2] += prev[3 * t + 2];
    }
    for (int t = threadIdx.x; t < I.nt2; t += blockDim.x) {
        v[3] += I.part2[2 * t + 1];
        v[4] = fmax(v[4], I.part2[2 * t]);
    }
    block_reduce_stats<5, 4>(v);
    if (threadIdx.x != 0) return;
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
        S.done = 1;
        S.stop_iter = kn;
    } else if (I.tol > 0.0 && gap <= I.tol) {
        S.converged = 1;
        S.done = 1;
        S.stop_iter = kn;
    }
}

// One workgroup per slot: the gap on the slot's check iterations (slots run
// by kb_persist take their gap there).
__global__ __launch_bounds__(1024) void kb_gap(const BInst* __restrict__ bi, BState* __restrict__ bs,
                                              const int64_t* __restrict__ dG, int64_t Gh, int ce) {
    const int64_t G = (dG ? *dG : Gh) + 1;
    const int gmod = (int)(G % ce);
    const BInst& I = bi[blockIdx.x];
    BState& S = bs[blockIdx.x];
    int64_t kn = 0;
    if (I.persist || !slot_live(I, S, G, &kn) || slot_phase(I, gmod) != 0) return;  // block-uniform
    slot_gap(I, S, kn);
}

// Small slots, one workgroup of 16 waves each: `iters` global iterations
// G0 + 1 .. G0 + iters (G0: the count when the call began) in one
// launch, the passes separated by workgroup barriers only.  Wave w takes
// tiles w, w + 16, ... of each pass: every tile computes exactly what it
// computes in the shared passes (the same tile functions, the same per-tile
// partials), and the gap uses the 1024-thread reduction of kb_gap, so the
// iterates and the stopping iteration are bit for bit the single path's.
// All writes a pass makes are read by the next pass of the same workgroup,
// which the barrier orders.
__global__ __launch_bounds__(1024) void kb_persist(const int32_t* __restrict__ slots, const BInst* __restrict__ bi,
                                                  BState* __restrict__ bs, const float* __restrict__ btab,
                                                  int64_t G0, int ce, int64_t iters) {
    __shared__ float lds[1024 / L1LS_WAVE][kTile * kMaxNnz];
    const int lane = threadIdx.x % L1LS_WAVE;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / L1LS_WAVE);
    constexpr int W = 1024 / L1LS_WAVE;
    const int slot = slots[blockIdx.x];
    const BInst& I = bi[slot];
    BState& S = bs[slot];
    const float Lf = (float)I.L, thr = (float)(I.tau / I.L);
    const int r2 = (int)((I.nt2 + W - 1) / W), r1 = (int)((I.nt1 + W - 1) / W);
    for (int64_t q = 1; q <= iters; ++q) {
        const int64_t G = G0 + q;
        int64_t kn = 0;
        if (!slot_live(I, S, G, &kn)) break;  // uniform: S.done is written before the last barrier
        const int ph = slot_phase(I, (int)(G % ce));
        const float bt = btab[kn - 1];
        for (int st = 0; st < r2; ++st)
            transpose_tile(I.csc_ptr, I.csc_row, I.csc_val, I.ry, I.x[(kn - 1) & 1], I.x[kn & 1], I.part2, I.n,
                           (int64_t)(st * W + wid) * kTile, bt, Lf, thr, ph == 0, true, lds[wid], lane);
        const float br = btab[kn];
        double* part1 = I.part1 + (size_t)(kn & 1) * I.nt1 * 3;
        for (int st = 0; st < r1; ++st)
            residual_tile(I.csr_ptr, I.csr_col, I.csr_val, I.x[kn & 1], I.b, I.rx, I.ry, part1, I.m,
                          (int64_t)(st * W + wid) * kTile, br, 0, ph == 0 || ph == ce - 1, true, lds[wid], lane);
        if (ph == 0) slot_gap(I, S, kn);
        __syncthreads();
    }
}

// End of a global iteration: the device's count G moves on (the kernels of
// the next iteration read it).
__global__ void kb_tick(int64_t* __restrict__ dG, int64_t by) { *dG += by; }

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

inline int64_t tiles_of(int64_t N) { return (N + kTile - 1) / kTile; }

// t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2 in the operation order of the
// single-instance driver, so both produce the same beta bits.
inline double next_t_host(double t) {
#pragma clang fp contract(off)
    return (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
}

}  // namespace

struct l1ls_batch {
    int32_t capacity = 0;
    size_t budget = 0, used = 0;
    hipStream_t stream = nullptr;
    l1ls_solve_opts o;
    int64_t G = 0;                            // global iterations enqueued
    std::vector<const l1ls_instance*> inst;   // per slot (nullptr: free)
    std::vector<BInst> hinst;
    std::vector<size_t> footprint;
    std::vector<void*> buf;                   // per-slot device block (iterates + partials)
    std::vector<char> retired;                // per slot: stopped (done or capped), out of the task tables
    // One-shot batches (l1ls_solve_fista_batched) carve the slot blocks from
    // one allocation: pool, pool_size bytes, pool_used taken so far; slots
    // in the pool are not freed one by one.
    char* pool = nullptr;
    size_t pool_size = 0, pool_used = 0;
    std::vector<char> pooled;
    BInst* dinst = nullptr;
    BState* dstate = nullptr;
    BTask* dt1 = nullptr;                     // residual-pass tasks of every slot (the first passes)
    BTask* dt1i = nullptr;                    // residual-pass tasks of the shared-pass slots (iterations)
    BTask* dt2 = nullptr;                     // transpose-pass tasks of the shared-pass slots
    int32_t cap1 = 0, cap1i = 0, cap2 = 0, nt1 = 0, nt1i = 0, nt2 = 0;
    int32_t* dsmall = nullptr;                // slots run by kb_persist
    int32_t nsmall = 0, capsmall = 0;
    hipStream_t side = nullptr;               // kb_persist runs here, beside the shared passes
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::vector<int32_t> steps;               // per slot: rounds per task (tile schedule)
    bool one = true;                          // every task has one round
    float* btab = nullptr;                    // beta_k, k = 0 .. nbeta-1
    int64_t nbeta = 0;
    bool tables_dirty = false, init_pending = false;
    DevAlloc* al = nullptr;                   // source of the slot blocks (nullptr: hipMalloc)
    int64_t* dG = nullptr;                    // device copy of G (the kernels read it; kb_tick advances it)
    // Graph mode (opts.graph): one check period of iterations captured once
    // per task table and replayed; cap_stream is the capture stream.
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int64_t graph_replays = 0;
    int64_t persist_rows = 0;                 // slots with m <= this run in kb_persist (0: none)
    DevArena arena;
};

namespace {

// Device bytes of a slot's own block: two x slots, r_x, r_y (FP32) and its
// FP64 partial sums.
size_t slot_fbytes(int64_t m, int64_t n) { return (((size_t)(2 * n + 2 * m) * sizeof(float) + 255) / 256) * 256; }

size_t slot_bytes(int64_t m, int64_t n) {
    return slot_fbytes(m, n) + (size_t)(6 * tiles_of(m) + 2 * tiles_of(n)) * sizeof(double);
}

void drop_graph(l1ls_batch* B);

// Slots of at most this many rows run their iterations in one workgroup
// (kb_persist) unless opts.persist_rows says otherwise.  Off by default: on
// the 256-instance workload the shared passes were faster (7,446 against
// 7,285 solves/s with m <= 4096 in one workgroup).
constexpr int64_t kPersistRows = 0;

// ---- tile-schedule autotuner ------------------------------------------------
// Rounds per task for a slot, by the size class ceil(log2(m)): unless the
// autotuner cache (tune.hpp, key batch_rounds/<class>) holds a choice, the
// first residual pass of the class's first slot (r = A x_0 - b, which the
// batch computes anyway) is timed with 1, 2, 4 and 8 rounds per task and the
// fastest is kept.
constexpr int kStepChoices[4] = {1, 2, 4, 8};

void push_tasks(std::vector<BTask>& out, int slot, int64_t rows, int32_t steps) {
    const int64_t per = (int64_t)4 * steps * kTile;  // rows per task
    for (int64_t r = 0; r < rows; r += per) out.push_back(BTask{slot, (int32_t)r, steps, 0});
}

// dinst must already hold the slot (admitted at B->G, init not yet run).
l1ls_status tune_steps(l1ls_batch* B, int slot, int32_t* best) {
    const BInst& h = B->hinst[slot];
    BTask* dt = nullptr;
    const int64_t max_tasks = (h.m + 4 * kTile - 1) / (4 * kTile);
    L1LS_TRY(B->arena.alloc(&dt, (size_t)max_tasks));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best_ms = 0.f;
    *best = 1;
    l1ls_status st = L1LS_OK;
    for (int c = 0; c < 4 && st == L1LS_OK; ++c) {
        std::vector<BTask> t;
        push_tasks(t, slot, h.m, kStepChoices[c]);
        if (hipMemcpyAsync(dt, t.data(), t.size() * sizeof(BTask), hipMemcpyHostToDevice, B->stream) != hipSuccess) {
            st = L1LS_E_HIP;
            break;
        }
        float ms = 0.f;
        for (int rep = 0; rep < 3; ++rep) {  // first launch warms up, two timed
            if (rep == 1) (void)hipEventRecord(e0, B->stream);
            if (kStepChoices[c] == 1)
                hipLaunchKernelGGL(kb_residual<true>, dim3((unsigned)t.size()), dim3(L1LS_BLOCK), 0, B->stream, dt,
                                   B->dinst, B->dstate, B->btab, (const int64_t*)nullptr, B->G, B->o.check_every, 1);
            else
                hipLaunchKernelGGL(kb_residual<false>, dim3((unsigned)t.size()), dim3(L1LS_BLOCK), 0, B->stream, dt,
                                   B->dinst, B->dstate, B->btab, (const int64_t*)nullptr, B->G, B->o.check_every, 1);
        }
        (void)hipEventRecord(e1, B->stream);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = L1LS_E_HIP;
            break;
        }
        if (c == 0 || ms < best_ms) {
            best_ms = ms;
            *best = kStepChoices[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

l1ls_status rebuild_tables(l1ls_batch* B) {
    HIP_TRY(hipMemcpyAsync(B->dinst, B->hinst.data(), B->capacity * sizeof(BInst), hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    std::vector<BTask> t1, t1i, t2;
    std::vector<int32_t> small;
    for (int s = 0; s < B->capacity; ++s) {
        if (!B->inst[s] || B->retired[s]) continue;
        const BInst& hi = B->hinst[s];
        if (B->steps[s] == 0) {
            if (B->o.tile_chunk > 0) {
                B->steps[s] = B->o.tile_chunk;
            } else {
                const std::string key = "batch_rounds/" + std::to_string(tune_size_class(hi.m));
                int32_t v = tune_lookup(key);
                if (v <= 0 && hi.admit == B->G) {  // a fresh slot: its first pass can be timed
                    L1LS_TRY(tune_steps(B, s, &v));
                    tune_store(key, v);
                }
                B->steps[s] = v > 0 ? v : 1;
            }
        }
        push_tasks(t1, s, hi.m, B->steps[s]);
        if (hi.persist) {
            small.push_back(s);
        } else {
            push_tasks(t1i, s, hi.m, B->steps[s]);
            push_tasks(t2, s, hi.n, B->steps[s]);
        }
    }
    auto grow = [&](BTask** d, int32_t* cap, size_t need) -> l1ls_status {
        if ((int32_t)need <= *cap) return L1LS_OK;
        *cap = std::max<int32_t>((int32_t)need, 2 * *cap);  // old tables stay in the arena until destroy
        return B->arena.alloc(d, (size_t)*cap);
    };
    L1LS_TRY(grow(&B->dt1, &B->cap1, t1.size()));
    L1LS_TRY(grow(&B->dt1i, &B->cap1i, t1i.size()));
    L1LS_TRY(grow(&B->dt2, &B->cap2, t2.size()));
    if ((int32_t)small.size() > B->capsmall) {
        B->capsmall = std::max<int32_t>((int32_t)small.size(), 2 * B->capsmall);
        L1LS_TRY(B->arena.alloc(&B->dsmall, (size_t)B->capsmall));
    }
    B->nt1 = (int32_t)t1.size();
    B->nt1i = (int32_t)t1i.size();
    B->nt2 = (int32_t)t2.size();
    B->nsmall = (int32_t)small.size();
    B->one = true;
    for (const BTask& t : t1) B->one = B->one && t.steps == 1;
    if (!t1.empty())
        HIP_TRY(hipMemcpyAsync(B->dt1, t1.data(), t1.size() * sizeof(BTask), hipMemcpyHostToDevice, B->stream));
    if (!t1i.empty())
        HIP_TRY(hipMemcpyAsync(B->dt1i, t1i.data(), t1i.size() * sizeof(BTask), hipMemcpyHostToDevice, B->stream));
    if (!t2.empty())
        HIP_TRY(hipMemcpyAsync(B->dt2, t2.data(), t2.size() * sizeof(BTask), hipMemcpyHostToDevice, B->stream));
    if (!small.empty())
        HIP_TRY(hipMemcpyAsync(B->dsmall, small.data(), small.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                               B->stream));
    // the copies read host vectors that go out of scope: wait for them
    HIP_TRY(hipStreamSynchronize(B->stream));
    B->tables_dirty = false;
    drop_graph(B);  // a captured period names the old task tables
    return L1LS_OK;
}

// beta_k = (t_k - 1) / t_{k+1} for k < need (beta_0 = 0, t_1 = 1), as FP32.
l1ls_status ensure_beta(l1ls_batch* B, int64_t need) {
    if (need <= B->nbeta) return L1LS_OK;
    const int64_t len = std::max<int64_t>(need, std::max<int64_t>(4096, 2 * B->nbeta));
    std::vector<float> h((size_t)len);
    h[0] = 0.f;
    double t = 1.0;
    for (int64_t k = 1; k < len; ++k) {
        const double tn = next_t_host(t);
        h[(size_t)k] = (float)((t - 1.0) / tn);
        t = tn;
    }
    float* d = nullptr;
    L1LS_TRY(B->arena.alloc(&d, (size_t)len));
    HIP_TRY(hipMemcpyAsync(d, h.data(), (size_t)len * sizeof(float), hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    B->btab = d;
    drop_graph(B);  // and the old beta table
    B->nbeta = len;
    return L1LS_OK;
}

l1ls_status run_init(l1ls_batch* B) {
    if (B->nt1 > 0) {
        if (B->one)
            hipLaunchKernelGGL(kb_residual<true>, dim3(B->nt1), dim3(L1LS_BLOCK), 0, B->stream, B->dt1, B->dinst,
                               B->dstate, B->btab, (const int64_t*)nullptr, B->G, B->o.check_every, 1);
        else
            hipLaunchKernelGGL(kb_residual<false>, dim3(B->nt1), dim3(L1LS_BLOCK), 0, B->stream, B->dt1, B->dinst,
                               B->dstate, B->btab, (const int64_t*)nullptr, B->G, B->o.check_every, 1);
        HIP_TRY(hipGetLastError());
    }
    B->init_pending = false;
    return L1LS_OK;
}

// Iteration a slot has reached: where it stopped, else its count capped.
int64_t slot_iterations(const l1ls_batch* B, int s, const BState& st) {
    if (st.done) return st.stop_iter;
    const BInst& h = B->hinst[s];
    const int64_t k = B->G - h.admit;
    return (h.max_iter > 0) ? std::min(k, h.max_iter) : k;
}

}  // namespace

// A slot's own device bytes (for admission estimates made before an
// instance exists).
size_t batch_slot_bytes(int64_t m, int64_t n) { return slot_bytes(m, n); }

// Take the slot blocks of a batch from `al` (set before any add; the
// batch's own tables stay on hipMalloc and are freed with the batch).
void batch_set_alloc(l1ls_batch* B, DevAlloc* al) { B->al = al; }

extern "C" l1ls_status l1ls_batch_create(int32_t capacity, size_t hbm_budget_bytes, const l1ls_solve_opts* opts,
                                         l1ls_batch** out) {
    if (!out || !opts || capacity < 1 || capacity > 65535) return L1LS_E_ARG;
    *out = nullptr;
    if (opts->precision != L1LS_F32 || opts->op != L1LS_OP_STORED) return L1LS_E_UNSUPPORTED;
    if (opts->check_every < 1 || !(opts->rel_gap_tol >= 0.0)) return L1LS_E_ARG;
    if (opts->tile_chunk < 0 || opts->tile_chunk > 64) return L1LS_E_ARG;
    if (opts->graph != 0 && opts->graph != 1) return L1LS_E_ARG;
    if (opts->persist_rows < -1) return L1LS_E_ARG;
    l1ls_batch* B = new l1ls_batch();
    B->capacity = capacity;
    B->budget = hbm_budget_bytes;
    B->stream = (hipStream_t)opts->stream;
    B->o = *opts;
    B->persist_rows = opts->persist_rows < 0 ? 0 : (opts->persist_rows > 0 ? opts->persist_rows : kPersistRows);
    B->inst.assign(capacity, nullptr);
    B->hinst.assign(capacity, BInst{});
    B->footprint.assign(capacity, 0);
    B->buf.assign(capacity, nullptr);
    B->retired.assign(capacity, 0);
    B->pooled.assign(capacity, 0);
    B->steps.assign(capacity, 0);
    auto fail = [&](l1ls_status s) {
        B->arena.release();
        delete B;
        return s;
    };
    l1ls_status st;
    if ((st = B->arena.alloc(&B->dinst, capacity)) != L1LS_OK) return fail(st);
    if ((st = B->arena.alloc(&B->dstate, capacity)) != L1LS_OK) return fail(st);
    if ((st = B->arena.alloc(&B->dG, 1)) != L1LS_OK) return fail(st);
    if ((st = ensure_beta(B, 4096)) != L1LS_OK) return fail(st);
    if (hipMemsetAsync(B->dG, 0, sizeof(int64_t), B->stream) != hipSuccess) return fail(L1LS_E_HIP);
    if (hipMemsetAsync(B->dstate, 0, capacity * sizeof(BState), B->stream) != hipSuccess) return fail(L1LS_E_HIP);
    if (hipMemsetAsync(B->dinst, 0, capacity * sizeof(BInst), B->stream) != hipSuccess) return fail(L1LS_E_HIP);
    if (hipStreamSynchronize(B->stream) != hipSuccess) return fail(L1LS_E_HIP);
    *out = B;
    return L1LS_OK;
}

extern "C" size_t l1ls_instance_footprint(const l1ls_instance* I) {
    if (!I) return 0;
    // stored FP32 CSR + CSC, FP64 copies if kept, vectors and tables, plus the
    // batch slot's iterates and partial sums
    size_t b = 0;
    if (I->csr_v32) b += (size_t)I->nnz * 16 + (size_t)(I->m + I->n + 2) * 4;
    if (I->csr_v64) b += (size_t)I->nnz * 16;
    b += (size_t)(I->m + I->n) * 48;
    return b + slot_bytes(I->m, I->n);
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
    const int64_t m = I->m, n = I->n;
    void* blk = nullptr;
    const size_t sb = slot_bytes(m, n);
    if (B->pool && B->pool_used + sb <= B->pool_size) {
        blk = B->pool + B->pool_used;
        B->pool_used += (sb + 255) / 256 * 256;
        B->pooled[slot] = 1;
    } else {
        L1LS_TRY(dev_alloc(B->al, &blk, sb));
        B->pooled[slot] = 0;
    }
    float* f = (float*)blk;
    hipLaunchKernelGGL(kb_zero, g1d(2 * n), dim3(L1LS_BLOCK), 0, B->stream, f, 2 * n);  // x_0 = x_{-1} = 0
    BInst& h = B->hinst[slot];
    h = BInst{};
    h.csr_ptr = I->csr_ptr;
    h.csr_col = I->csr_col;
    h.csr_val = I->csr_v32;
    h.csc_ptr = I->csc_ptr;
    h.csc_row = I->csc_row;
    h.csc_val = I->csc_v32;
    h.b = I->b32_op;
    h.x[0] = f;
    h.x[1] = f + n;
    h.rx = f + 2 * n;
    h.ry = f + 2 * n + m;
    h.part1 = (double*)((char*)blk + slot_fbytes(m, n));
    h.part2 = h.part1 + 6 * tiles_of(m);
    h.m = m;
    h.n = n;
    h.admit = B->G;
    h.max_iter = max_iter > 0 ? max_iter : 0;
    h.tau = tau;
    h.L = I->L;
    h.tol = rel_gap_tol >= 0.0 ? rel_gap_tol : B->o.rel_gap_tol;
    h.nt1 = (int32_t)tiles_of(m);
    h.nt2 = (int32_t)tiles_of(n);
    h.check_every = B->o.check_every;
    h.admit_mod = (int32_t)(B->G % B->o.check_every);
    h.active = 1;
    h.persist = (B->persist_rows > 0 && m <= B->persist_rows) ? 1 : 0;
    B->inst[slot] = I;
    B->buf[slot] = blk;
    B->footprint[slot] = fp;
    B->used += fp;
    B->retired[slot] = 0;
    // a fresh state (stream-ordered before the slot's first pass)
    HIP_TRY(hipMemsetAsync(B->dstate + slot, 0, sizeof(BState), B->stream));
    HIP_TRY(hipGetLastError());
    B->tables_dirty = true;
    B->init_pending = true;
    *slot_out = slot;
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_batch_add(l1ls_batch* B, const l1ls_instance* I, double tau, int32_t* slot_out) {
    return l1ls_batch_add_ex(B, I, tau, -1.0, 0, slot_out);
}

namespace {

// The kernels of one global iteration of the shared-pass slots on `s`:
// transpose pass, residual pass, the gap kernel (when `gap`; it returns at
// once for slots not at a check iteration) and the step of the device's G.
void enqueue_iteration(l1ls_batch* B, hipStream_t s, bool gap, bool graph) {
    const int ce = B->o.check_every;
    // graph replays read the count from the device (kb_tick advances it);
    // launched iterations take it as an argument (host G before the step)
    const int64_t* dG = graph ? B->dG : nullptr;
    const int64_t Gh = B->G;
    if (B->nt1i > 0) {
        if (B->one) {
            hipLaunchKernelGGL(kb_transpose<true>, dim3(B->nt2), dim3(L1LS_BLOCK), 0, s, B->dt2, B->dinst,
                               B->dstate, B->btab, dG, Gh, ce);
            hipLaunchKernelGGL(kb_residual<true>, dim3(B->nt1i), dim3(L1LS_BLOCK), 0, s, B->dt1i, B->dinst,
                               B->dstate, B->btab, dG, Gh, ce, 0);
        } else {
            hipLaunchKernelGGL(kb_transpose<false>, dim3(B->nt2), dim3(L1LS_BLOCK), 0, s, B->dt2, B->dinst,
                               B->dstate, B->btab, dG, Gh, ce);
            hipLaunchKernelGGL(kb_residual<false>, dim3(B->nt1i), dim3(L1LS_BLOCK), 0, s, B->dt1i, B->dinst,
                               B->dstate, B->btab, dG, Gh, ce, 0);
        }
        if (gap) hipLaunchKernelGGL(kb_gap, dim3(B->capacity), dim3(1024), 0, s, B->dinst, B->dstate, dG, Gh, ce);
    }
    if (graph) hipLaunchKernelGGL(kb_tick, dim3(1), dim3(1), 0, s, B->dG, (int64_t)1);
}

void drop_graph(l1ls_batch* B) {
    if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->gexec = nullptr;
    B->graph = nullptr;
}

// Capture one check period of iterations (every one with the gap kernel:
// which iterations are check iterations moves with G) on the capture stream.
// Kernel arguments are the task tables, the beta table and the device G, so
// the graph stays valid until one of those is replaced.
l1ls_status capture_period(l1ls_batch* B) {
    drop_graph(B);
    if (!B->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int q = 0; q < B->o.check_every; ++q) enqueue_iteration(B, B->cap_stream, true, true);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(B->cap_stream, &g);
    if (e != hipSuccess || !g) return L1LS_E_HIP;
    B->graph = g;
    HIP_TRY(hipGraphInstantiate(&B->gexec, B->graph, nullptr, nullptr, 0));
    return L1LS_OK;
}

}  // namespace

extern "C" l1ls_status l1ls_batch_iterate(l1ls_batch* B, int64_t iters) {
    if (!B || iters < 0) return L1LS_E_ARG;
    if (B->tables_dirty) L1LS_TRY(rebuild_tables(B));
    if (B->init_pending) L1LS_TRY(run_init(B));
    if (iters == 0) return L1LS_OK;
    const bool graph = B->o.graph != 0;
    if (B->nt1 == 0) {  // nothing resident: the count still advances (on the device too in graph mode)
        if (graph) hipLaunchKernelGGL(kb_tick, dim3(1), dim3(1), 0, B->stream, B->dG, iters);
        B->G += iters;
        HIP_TRY(hipGetLastError());
        return L1LS_OK;
    }
    // the beta table must reach the largest k any slot can take; the gap
    // kernel runs on the G at which some slot's k is a multiple of check_every
    const int64_t ce = B->o.check_every;
    int64_t oldest = B->G;
    std::vector<char> phase((size_t)ce, 0);
    for (int s = 0; s < B->capacity; ++s)
        if (B->inst[s]) {
            oldest = std::min(oldest, B->hinst[s].admit);
            phase[(size_t)(B->hinst[s].admit % ce)] = 1;
        }
    L1LS_TRY(ensure_beta(B, B->G + iters - oldest + 2));
    if (B->nsmall > 0) {
        // the small slots: all `iters` iterations in one launch on the side
        // stream, beside the shared passes; the stream joins at the end
        if (!B->side) {
            HIP_TRY(hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
            HIP_TRY(hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming));
        }
        HIP_TRY(hipEventRecord(B->ev_fork, B->stream));
        HIP_TRY(hipStreamWaitEvent(B->side, B->ev_fork, 0));
        hipLaunchKernelGGL(kb_persist, dim3(B->nsmall), dim3(1024), 0, B->side, (const int32_t*)B->dsmall, B->dinst,
                           B->dstate, B->btab, B->G, (int)ce, iters);
        HIP_TRY(hipEventRecord(B->ev_join, B->side));
    }
    if (graph && B->nt1i > 0) {
        // whole check periods by graph replay, the rest launched one by one
        // (the device count follows G in graph mode)
        while (iters >= ce) {
            if (!B->gexec) L1LS_TRY(capture_period(B));
            HIP_TRY(hipGraphLaunch(B->gexec, B->stream));
            B->G += ce;
            B->graph_replays += 1;
            iters -= ce;
        }
    }
    if (B->nt1i > 0) {
        for (int64_t q = 0; q < iters; ++q) {
            const int gmod = (int)((B->G + 1) % ce);
            enqueue_iteration(B, B->stream, phase[(size_t)gmod] != 0, graph);
            ++B->G;
        }
    } else {
        if (graph) hipLaunchKernelGGL(kb_tick, dim3(1), dim3(1), 0, B->stream, B->dG, iters);
        B->G += iters;
    }
    if (B->nsmall > 0) HIP_TRY(hipStreamWaitEvent(B->stream, B->ev_join, 0));
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
        const BInst& h = B->hinst[s];
        r.iterations = slot_iterations(B, s, st[s]);
        r.primal = st[s].P;
        r.dual = st[s].D;
        r.rel_gap = st[s].gap;
        r.converged = st[s].converged ? 1 : (st[s].nonfinite ? -1 : 0);
        r.rel_err = -1.0;
        const bool capped = h.max_iter > 0 && r.iterations >= h.max_iter;
        if (!st[s].done && !capped) {
            ++act;
        } else if (!B->retired[s]) {
            // a stopped slot's passes do nothing: drop its tasks from the
            // shared launches (its iterate and state stay until remove)
            B->retired[s] = 1;
            B->tables_dirty = true;
        }
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
    const int64_t k = slot_iterations(B, slot, st);
    hipLaunchKernelGGL(kb_to_f64_perm, g1d(I->n), dim3(L1LS_BLOCK), 0, B->stream, B->hinst[slot].x[k & 1], x_out,
                       I->op_col_pos, I->n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(B->stream));
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_batch_remove(l1ls_batch* B, int32_t slot) {
    if (!B || slot < 0 || slot >= B->capacity || !B->inst[slot]) return L1LS_E_ARG;
    HIP_TRY(hipStreamSynchronize(B->stream));
    if (!B->pooled[slot]) dev_free(B->al, B->buf[slot], slot_bytes(B->hinst[slot].m, B->hinst[slot].n));
    B->pooled[slot] = 0;
    B->retired[slot] = 0;
    B->buf[slot] = nullptr;
    B->used -= B->footprint[slot];
    B->footprint[slot] = 0;
    B->inst[slot] = nullptr;
    B->hinst[slot] = BInst{};
    B->steps[slot] = 0;
    B->tables_dirty = true;
    return L1LS_OK;
}

extern "C" void l1ls_batch_destroy(l1ls_batch* B) {
    if (!B) return;
    (void)hipStreamSynchronize(B->stream);
    if (B->side) (void)hipStreamSynchronize(B->side);
    (void)hipDeviceSynchronize();  // one wait for all the slot blocks
    for (int s = 0; s < B->capacity; ++s)
        if (B->buf[s] && !B->pooled[s]) dev_free(B->al, B->buf[s], slot_bytes(B->hinst[s].m, B->hinst[s].n), true);
    if (B->pool) dev_free(B->al, B->pool, B->pool_size, true);
    drop_graph(B);
    if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
    if (B->side) (void)hipStreamSynchronize(B->side);
    if (B->side) (void)hipStreamDestroy(B->side);
    if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
    if (B->ev_join) (void)hipEventDestroy(B->ev_join);
    B->arena.release();
    delete B;
}

extern "C" l1ls_status l1ls_solve_fista_batched(const l1ls_instance* const* insts, const double* taus, int32_t count,
                                                const l1ls_solve_opts* opts, double* const* x_outs,
                                                l1ls_report* reports) {
    if (!insts || !opts || !x_outs || !reports || count < 1) return L1LS_E_ARG;
    for (int q = 0; q < count; ++q)
        if (!insts[q] || !x_outs[q]) return L1LS_E_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    l1ls_batch* B = nullptr;
    L1LS_TRY(l1ls_batch_create(count, 0, opts, &B));
    // every slot block from one allocation
    size_t total = 0;
    for (int q = 0; q < count; ++q) total += (slot_bytes(insts[q]->m, insts[q]->n) + 255) / 256 * 256;
    l1ls_status st = dev_alloc(B->al, (void**)&B->pool, total);
    if (st == L1LS_OK) B->pool_size = total;
    std::vector<int32_t> slot(count, -1);
    for (int q = 0; q < count && st == L1LS_OK; ++q)
        st = l1ls_batch_add_ex(B, insts[q], taus ? taus[q] : 0.0, -1.0, opts->max_iter, &slot[q]);
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
    // every result from the states just polled, one wait at the end
    bool all = true;
    for (int q = 0; q < count && st == L1LS_OK; ++q) {
        const int s = slot[q];
        const l1ls_instance* I = B->inst[s];
        const int64_t k = rep[s].iterations;
        hipLaunchKernelGGL(kb_to_f64_perm, g1d(I->n), dim3(L1LS_BLOCK), 0, B->stream, B->hinst[s].x[k & 1],
                           x_outs[q], I->op_col_pos, I->n);
        reports[q] = rep[s];
        all = all && reports[q].converged == 1;
    }
    if (st == L1LS_OK && (hipGetLastError() != hipSuccess || hipStreamSynchronize(B->stream) != hipSuccess))
        st = L1LS_E_HIP;
    l1ls_batch_destroy(B);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int q = 0; q < count; ++q) reports[q].seconds = secs;
    if (st != L1LS_OK) return st;
    return all ? L1LS_OK : L1LS_NOT_CONVERGED;
}
