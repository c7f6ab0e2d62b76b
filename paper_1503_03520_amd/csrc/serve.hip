// Serving scheduler: continuous batching of l1-LS solve requests on one GPU.
//
// Requests (instance parameters of Procedure IGen, section 3.1, and a
// relative-gap tolerance) wait in one FIFO queue per size class (n < 2^14,
// n < 2^18, larger).  Resident requests live in one batch per class, each
// on its own stream, so a small instance advances at its own iteration rate
// alongside a large one instead of in lockstep with it.  The largest class
// holds one request at a time: its iterations already saturate HBM, so
// sharing the device among several would only delay the first to finish.
// Each tick:
//  1. enqueue iterations of every class with residents: the slowest class
//     runs at least `iters_per_tick` iterations (and the tick at least
//     kMinTickS), the others as many as fit the same time (estimated from
//     bytes per iteration with a launch floor), in multiples of the
//     gap-check period;
//  2. admission, while those run: repeatedly take the oldest class-queue
//     head that fits (a slot free, its class below its resident limit, its
//     footprint, estimated before generation from the bound of 4^rounds
//     nonzeros per column of A = Q Sigma G^T, eq. (16), within the HBM
//     budget), generate its instance on the device (own stream) and add it
//     to its class's batch; it starts iterating in the next tick;
//  3. retire the slots whose gap test passed, whose iterate went
//     non-finite, or which reached their cap: copy the iterate to a result
//     buffer, free the slot and the instance.
// A request's arithmetic depends only on its own instance and iteration
// count (the batch's per-slot independence), so a result is the same in any
// mix, any class schedule and any tick length.
//
// Requests flagged for an FP64 finish leave the batch into a queue served
// by a worker thread of their size class, on its own stream: FP64 gap of the
// iterate, and the FP64 polish of the reduced problem (13) (section 3.2)
// when the gap misses the tolerance.  The tick loop never waits for a
// polish, and a small request's certificate never waits for a large one's
// polish.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"

size_t batch_slot_bytes(int64_t m, int64_t n);
void batch_set_alloc(l1ls_batch* B, DevAlloc* al);
l1ls_status generate_with(int64_t m, int64_t n, double kappa, int64_t s, double tau, uint64_t seed,
                          const l1ls_gen_opts* opts, DevAlloc* al, l1ls_instance** out);
void free_idle_instance(l1ls_instance* I);
l1ls_status gap_fp64(const l1ls_instance* I, double tau, const double* x, double* P, double* D, double* gap,
                     hipStream_t s, DevAlloc* al = nullptr);
l1ls_status polish_fp64(const l1ls_instance* I, double tau, double* x_dev, hipStream_t stream, int* rounds_out,
                        int64_t* pcg_iters_out, double support_tol, DevAlloc* al = nullptr);

namespace {

using ServeClock = std::chrono::steady_clock;

constexpr int kClasses = 3;
constexpr double kIterFloorS = 9e-6;   // launch-bound floor of one batched iteration
constexpr double kBytesPerS = 4.5e12;  // sustained rate of the SpMV pair
constexpr double kMinTickS = 1e-3;     // shortest tick (host work per tick is ~0.1 ms)
constexpr int kMaxTickMultiple = 64;   // cap on a class's iterations per tick, in iters_per_tick

constexpr int32_t kClassLimit[kClasses] = {65535, 65535, 1};  // residents per class

int class_of(int64_t n) { return n < (1 << 14) ? 0 : (n < (1 << 18) ? 1 : 2); }

// Algorithmic bytes of one FISTA iteration of an instance (FP32, int32).
double iter_bytes(int64_t m, int64_t n, int64_t nnz) { return 16.0 * nnz + 24.0 * m + 20.0 * n; }

// Caching device allocator of a server.  hipFree waits for every stream of
// the device, so a free in the serving loop would stall the other size
// classes and workers; instead freed blocks go to per-size free lists
// (sizes rounded up to a quarter octave, at most 25% slack) and are reused.
// Cached bytes beyond `cap` go back to the library's device-memory source
// (l1ls_set_allocator); everything goes back when the server is destroyed.
class ServePool : public DevAlloc {
   public:
    explicit ServePool(size_t cap) : cap_(cap) {}
    ~ServePool() override { trim(0); }
    static size_t round(size_t b) {
        if (b <= 4096) return 4096;
        int e = 63 - __builtin_clzll((unsigned long long)b);  // 2^e <= b < 2^(e+1)
        const size_t q = (size_t)1 << (e - 2);                  // quarter octave
        return ((b + q - 1) / q) * q;
    }
    l1ls_status alloc(void** p, size_t bytes) override {
        const size_t r = round(bytes);
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.find(r);
            if (it != free_.end() && !it->second.empty()) {
                *p = it->second.back();
                it->second.pop_back();
                cached_ -= r;
                return L1LS_OK;
            }
        }
        if (lib_alloc(p, r) != L1LS_OK) {
            trim(0);  // give the cache back and try once more
            if (lib_alloc(p, r) != L1LS_OK) return L1LS_E_NOMEM;
        }
        return L1LS_OK;
    }
    void free(void* p, size_t bytes) override {
        if (!p) return;
        const size_t r = round(bytes);
        std::lock_guard<std::mutex> lk(mu_);
        free_[r].push_back(p);
        cached_ += r;
        if (cached_ > cap_) trim_locked(cap_ / 2);
    }
    void trim(size_t keep) {
        std::lock_guard<std::mutex> lk(mu_);
        trim_locked(keep);
    }

   private:
    void trim_locked(size_t keep) {  // largest blocks first
        for (auto it = free_.rbegin(); it != free_.rend() && cached_ > keep; ++it)
            while (!it->second.empty() && cached_ > keep) {
                lib_free(it->second.back(), it->first);
                it->second.pop_back();
                cached_ -= it->first;
            }
    }
    std::mutex mu_;
    std::map<size_t, std::vector<void*>> free_;
    size_t cached_ = 0, cap_;
};

struct ServeReq {
    int64_t id;
    l1ls_request r;
    ServeClock::time_point submitted;
};

struct ServeSlot {
    int64_t id = -1;
    l1ls_instance* inst = nullptr;
    int64_t max_iter = 0;
    size_t est = 0;
    double bytes = 0.0;
    double tau = 0.0, tol = 0.0;
    bool finish = false;
    ServeClock::time_point submitted;
};

struct ServeDone {
    double* x = nullptr;  // n FP64 on the device
    int64_t n = 0;
    l1ls_report rep;
};

struct FinishJob {  // a retired FP64-finish request waiting for its worker
    int64_t id = -1;
    int cls = 0;
    l1ls_instance* inst = nullptr;
    ServeDone d;
    double tau = 0.0, tol = 0.0;
    size_t est = 0;
    ServeClock::time_point submitted;
};

struct ServeClass {
    l1ls_batch* batch = nullptr;
    hipStream_t stream = nullptr;
    std::vector<ServeSlot> slots;  // by batch slot
    int32_t resident = 0;
    double bytes = 0.0;  // per-iteration bytes of the residents
};

}  // namespace

struct l1ls_server {
    int32_t max_slots = 0, iters_per_tick = 0, check_every = 0;
    int device = 0;
    size_t budget = 0;
    hipStream_t stream = nullptr;  // caller's stream: result copies
    hipStream_t gen_stream = nullptr;
    hipStream_t fin_stream[kClasses] = {nullptr, nullptr, nullptr};
    ServeClass cls[kClasses];
    int64_t next_id = 0;
    std::deque<ServeReq> queue[kClasses];
    // shared with the finishing worker (under mu)
    std::mutex mu;
    std::condition_variable cv;
    size_t used = 0;
    std::deque<FinishJob> jobs[kClasses];
    int32_t finishing = 0;  // jobs queued or running
    bool stop = false;
    l1ls_status worker_status = L1LS_OK;
    std::unordered_map<int64_t, ServeDone> done;
    std::vector<int64_t> fresh;  // retired since the last l1ls_server_completed call
    std::thread worker[kClasses];
    ServePool* pool = nullptr;
};

namespace {

// The terms of l1ls_instance_footprint for an FP32-only instance, with nnz
// at its bound (each Givens stage at most doubles a column's support).
size_t estimate_footprint(const l1ls_request& r) {
    const size_t nnz = (size_t)r.n * (r.rounds >= 2 ? 16 : 4);
    const size_t f64 = (r.flags & L1LS_REQ_FP64_FINISH) ? nnz * 16 : 0;
    return nnz * 16 + f64 + (size_t)(r.m + r.n + 2) * 4 + (size_t)(r.m + r.n) * 48 + batch_slot_bytes(r.m, r.n);
}

bool valid_request(const l1ls_request& r) {
    return r.n >= 2 && r.m >= r.n && r.m % 2 == 0 && r.n % 2 == 0 && r.m < ((int64_t)1 << 31) && r.s >= 0 &&
           r.s <= r.n && r.kappa >= 1.0 && is_finite(r.kappa) && r.tau > 0.0 && is_finite(r.tau) &&
           (r.rounds == 1 || r.rounds == 2) && r.rel_gap_tol > 0.0 && r.max_iter > 0 &&
           (r.flags & ~L1LS_REQ_FP64_FINISH) == 0;
}

void destroy_streams(l1ls_server* S) {
    for (ServeClass& c : S->cls)
        if (c.stream) (void)hipStreamDestroy(c.stream);
    if (S->gen_stream) (void)hipStreamDestroy(S->gen_stream);
    for (hipStream_t& f : S->fin_stream)
        if (f) (void)hipStreamDestroy(f);
}

// Requests holding a slot or waiting for / in the finishing worker (call
// with mu held or from the tick thread, which alone changes the slots).
int32_t total_resident(const l1ls_server* S) {
    int32_t r = S->finishing;
    for (const ServeClass& c : S->cls) r += c.resident;
    return r;
}

// The finishing worker of size class c: FP64 gap, polish when the gap
// misses the tolerance, FP64 gap again; then the result joins the completed
// ones.
void finish_worker(l1ls_server* S, int c) {
    (void)hipSetDevice(S->device);
    hipStream_t fs = S->fin_stream[c];
    for (;;) {
        FinishJob j;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [S, c] { return S->stop || !S->jobs[c].empty(); });
            if (S->jobs[c].empty()) return;  // stop requested and nothing left
            j = S->jobs[c].front();
            S->jobs[c].pop_front();
        }
        double P = 0.0, D = 0.0, gap = INFINITY;
        int rounds = 0;
        int64_t pcg = 0;
        l1ls_status st = gap_fp64(j.inst, j.tau, j.d.x, &P, &D, &gap, fs, S->pool);
        if (st == L1LS_OK && !(gap <= j.tol)) {
            st = polish_fp64(j.inst, j.tau, j.d.x, fs, &rounds, &pcg, 0.0, S->pool);
            if (st == L1LS_OK) st = gap_fp64(j.inst, j.tau, j.d.x, &P, &D, &gap, fs, S->pool);
        }
        j.d.rep.primal = P;
        j.d.rep.dual = D;
        j.d.rep.rel_gap = gap;
        j.d.rep.polish_rounds = rounds;
        j.d.rep.inner = pcg;
        j.d.rep.converged = (st == L1LS_OK && gap <= j.tol) ? 1 : (j.d.rep.converged < 0 ? -1 : 0);
        j.d.rep.seconds = std::chrono::duration<double>(ServeClock::now() - j.submitted).count();
        (void)hipStreamSynchronize(fs);
        free_idle_instance(j.inst);
        std::lock_guard<std::mutex> lk(S->mu);
        if (st != L1LS_OK) S->worker_status = st;
        S->used -= j.est;
        S->finishing -= 1;
        S->done[j.id] = j.d;
        S->fresh.push_back(j.id);
    }
}

void stop_workers(l1ls_server* S) {
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    for (std::thread& w : S->worker)
        if (w.joinable()) w.join();
}

}  // namespace

extern "C" l1ls_status l1ls_server_create(int32_t max_slots, size_t hbm_budget_bytes, int32_t iters_per_tick,
                                          int32_t check_every, void* stream, l1ls_server** out) {
    if (!out || max_slots < 1 || max_slots > 65535 || iters_per_tick < 1 || check_every < 1) return L1LS_E_ARG;
    *out = nullptr;
    l1ls_server* S = new l1ls_server();
    S->max_slots = max_slots;
    S->iters_per_tick = iters_per_tick;
    S->check_every = check_every;
    S->budget = hbm_budget_bytes;
    S->stream = (hipStream_t)stream;
    // cached free blocks are capped at a quarter of the budget (8 GiB without one)
    S->pool = new ServePool(hbm_budget_bytes ? hbm_budget_bytes / 4 : ((size_t)8 << 30));
    auto fail = [&](l1ls_status st) {
        for (ServeClass& c : S->cls)
            if (c.batch) l1ls_batch_destroy(c.batch);
        delete S->pool;
        destroy_streams(S);
        delete S;
        return st;
    };
    if (hipGetDevice(&S->device) != hipSuccess) return fail(L1LS_E_HIP);
    if (hipStreamCreateWithFlags(&S->gen_stream, hipStreamNonBlocking) != hipSuccess) return fail(L1LS_E_HIP);
    for (hipStream_t& f : S->fin_stream)
        if (hipStreamCreateWithFlags(&f, hipStreamNonBlocking) != hipSuccess) return fail(L1LS_E_HIP);
    for (ServeClass& c : S->cls) {
        if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess) return fail(L1LS_E_HIP);
        l1ls_solve_opts o;
        l1ls_solve_opts_default(&o);
        o.precision = L1LS_F32;
        o.op = L1LS_OP_STORED;
        o.check_every = check_every;
        o.rel_gap_tol = 1e-6;  // every slot gets its request's own tolerance
        o.stream = c.stream;
        l1ls_status st = l1ls_batch_create(max_slots, 0, &o, &c.batch);
        if (st != L1LS_OK) return fail(st);
        batch_set_alloc(c.batch, S->pool);
        c.slots.assign(max_slots, ServeSlot{});
    }
    try {
        for (int c = 0; c < kClasses; ++c) S->worker[c] = std::thread(finish_worker, S, c);
    } catch (...) {
        stop_workers(S);
        return fail(L1LS_E_STATE);
    }
    *out = S;
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_server_submit(l1ls_server* S, const l1ls_request* r, int64_t* id_out) {
    if (!S || !r || !id_out || !valid_request(*r)) return L1LS_E_ARG;
    if (S->budget && estimate_footprint(*r) > S->budget) return L1LS_E_NOMEM;  // could never be admitted
    ServeReq q;
    q.id = S->next_id++;
    q.r = *r;
    q.submitted = ServeClock::now();
    S->queue[class_of(r->n)].push_back(q);
    *id_out = q.id;
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_server_tick(l1ls_server* S, int32_t* admitted, int32_t* completed) {
    if (!S) return L1LS_E_ARG;
    int32_t na = 0, nc = 0;
    const int64_t ce = S->check_every;
    // 1. iterations of the resident classes, sized to one common tick length
    double tmax = 0.0;
    double tc[kClasses];
    for (int c = 0; c < kClasses; ++c) {
        tc[c] = std::max(kIterFloorS, S->cls[c].bytes / kBytesPerS);
        if (S->cls[c].resident) tmax = std::max(tmax, tc[c]);
    }
    const double tick_s = std::max(kMinTickS, tmax * S->iters_per_tick);
    const int64_t lo = ((S->iters_per_tick + ce - 1) / ce) * ce;
    const int64_t hi = std::max<int64_t>(lo, ((int64_t)kMaxTickMultiple * S->iters_per_tick / ce) * ce);
    for (int c = 0; c < kClasses; ++c) {
        ServeClass& C = S->cls[c];
        if (!C.resident) continue;
        int64_t it = (int64_t)std::floor(tick_s / tc[c] / (double)ce) * ce;
        it = std::min(std::max(it, lo), hi);
        L1LS_TRY(l1ls_batch_iterate(C.batch, it));
    }
    // 2. admission: the oldest class-queue head that fits, repeatedly, while those run
    for (;;) {
        int pick = -1;
        for (int c = 0; c < kClasses; ++c) {
            if (S->queue[c].empty() || S->cls[c].resident >= kClassLimit[c]) continue;
            const ServeReq& h = S->queue[c].front();
            std::lock_guard<std::mutex> lk(S->mu);
            if (total_resident(S) >= S->max_slots) continue;
            if (S->budget && S->used + estimate_footprint(h.r) > S->budget) continue;
            if (pick < 0 || h.id < S->queue[pick].front().id) pick = c;
        }
        if (pick < 0) break;
        const ServeReq q = S->queue[pick].front();
        const l1ls_request& r = q.r;
        ServeClass& C = S->cls[pick];
        l1ls_gen_opts go;
        go.rounds = r.rounds;
        go.storage = (r.flags & L1LS_REQ_FP64_FINISH) ? (L1LS_STORE_F32 | L1LS_STORE_F64) : L1LS_STORE_F32;
        go.stream = S->gen_stream;
        go.layout = L1LS_LAYOUT_STAGE;
        l1ls_instance* inst = nullptr;
        L1LS_TRY(generate_with(r.m, r.n, r.kappa, r.s, r.tau, r.seed, &go, S->pool, &inst));
        int32_t bslot = -1;
        l1ls_status st = l1ls_batch_add_ex(C.batch, inst, r.tau, r.rel_gap_tol, r.max_iter, &bslot);
        if (st != L1LS_OK) {
            free_idle_instance(inst);  // generation has finished and nothing else used it
            return st;
        }
        const size_t fp = estimate_footprint(r);
        ServeSlot& sl = C.slots[bslot];
        sl.id = q.id;
        sl.inst = inst;
        sl.max_iter = r.max_iter;
        sl.est = fp;
        sl.bytes = iter_bytes(inst->m, inst->n, inst->nnz);
        sl.tau = r.tau;
        sl.tol = r.rel_gap_tol;
        sl.finish = (r.flags & L1LS_REQ_FP64_FINISH) != 0;
        sl.submitted = q.submitted;
        C.resident += 1;
        C.bytes += sl.bytes;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->used += fp;
        }
        S->queue[pick].pop_front();
        ++na;
    }
    // 3. retirement
    std::vector<l1ls_report> reps(S->max_slots);
    for (ServeClass& C : S->cls) {
        if (!C.resident) continue;
        L1LS_TRY(l1ls_batch_poll(C.batch, reps.data(), nullptr));
        for (int q = 0; q < S->max_slots; ++q) {
            ServeSlot& sl = C.slots[q];
            if (sl.id < 0) continue;
            const l1ls_report& rp = reps[q];
            if (rp.converged == 0 && rp.iterations < sl.max_iter) continue;  // still iterating
            ServeDone d;
            d.n = sl.inst->n;
            d.rep = rp;
            void* p = nullptr;
            L1LS_TRY(S->pool->alloc(&p, d.n * sizeof(double)));
            d.x = (double*)p;
            l1ls_status st = l1ls_batch_get_x(C.batch, q, d.x);  // synchronises the class stream
            if (st == L1LS_OK) st = l1ls_batch_remove(C.batch, q);
            if (st != L1LS_OK) {
                S->pool->free(p, d.n * sizeof(double));
                return st;
            }
            C.resident -= 1;
            C.bytes -= sl.bytes;
            if (C.resident == 0) C.bytes = 0.0;
            if (sl.finish) {  // to the worker; it frees the instance and releases the budget
                FinishJob j;
                j.id = sl.id;
                j.cls = (int)(&C - S->cls);
                j.inst = sl.inst;
                j.d = d;
                j.tau = sl.tau;
                j.tol = sl.tol;
                j.est = sl.est;
                j.submitted = sl.submitted;
                {
                    std::lock_guard<std::mutex> lk(S->mu);
                    S->finishing += 1;
                    S->jobs[j.cls].push_back(j);
                }
                S->cv.notify_all();
            } else {
                d.rep.seconds = std::chrono::duration<double>(ServeClock::now() - sl.submitted).count();
                free_idle_instance(sl.inst);  // its class stream was synchronised by the removal
                std::lock_guard<std::mutex> lk(S->mu);
                S->used -= sl.est;
                S->done[sl.id] = d;
                S->fresh.push_back(sl.id);
                ++nc;
            }
            sl = ServeSlot{};
        }
    }
    if (admitted) *admitted = na;
    if (completed) *completed = nc;
    std::lock_guard<std::mutex> lk(S->mu);
    return S->worker_status;
}

extern "C" int32_t l1ls_server_completed(l1ls_server* S, int64_t* ids, int32_t cap) {
    if (!S || !ids || cap < 1) return 0;
    std::lock_guard<std::mutex> lk(S->mu);
    const int32_t k = (int32_t)std::min<size_t>((size_t)cap, S->fresh.size());
    for (int32_t q = 0; q < k; ++q) ids[q] = S->fresh[q];
    S->fresh.erase(S->fresh.begin(), S->fresh.begin() + k);
    return k;
}

extern "C" l1ls_status l1ls_server_take(l1ls_server* S, int64_t id, double* x_out_dev, l1ls_report* rep) {
    if (!S) return L1LS_E_ARG;
    ServeDone d;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->done.find(id);
        if (it == S->done.end()) return L1LS_E_STATE;
        d = it->second;
        S->done.erase(it);
    }
    l1ls_status st = L1LS_OK;
    if (x_out_dev &&
        hipMemcpyAsync(x_out_dev, d.x, d.n * sizeof(double), hipMemcpyDeviceToDevice, S->stream) != hipSuccess)
        st = L1LS_E_HIP;
    if (hipStreamSynchronize(S->stream) != hipSuccess) st = L1LS_E_HIP;
    if (rep) *rep = d.rep;
    S->pool->free(d.x, d.n * sizeof(double));
    return st;
}

extern "C" l1ls_status l1ls_server_stats(l1ls_server* S, int32_t* queued, int32_t* resident, size_t* used_bytes) {
    if (!S) return L1LS_E_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    if (queued) {
        size_t qn = 0;
        for (const auto& q : S->queue) qn += q.size();
        *queued = (int32_t)qn;
    }
    if (resident) *resident = total_resident(S);
    if (used_bytes) *used_bytes = S->used;
    return L1LS_OK;
}

extern "C" size_t l1ls_request_footprint(const l1ls_request* r) {
    return (r && valid_request(*r)) ? estimate_footprint(*r) : 0;
}

extern "C" void l1ls_server_destroy(l1ls_server* S) {
    if (!S) return;
    stop_workers(S);  // finish the queued jobs first
    for (ServeClass& C : S->cls)
        if (C.stream) (void)hipStreamSynchronize(C.stream);
    if (S->gen_stream) (void)hipStreamSynchronize(S->gen_stream);
    for (ServeClass& C : S->cls) {
        for (ServeSlot& s : C.slots)
            if (s.inst) free_idle_instance(s.inst);
        if (C.batch) l1ls_batch_destroy(C.batch);
    }
    for (auto& kv : S->done) S->pool->free(kv.second.x, kv.second.n * sizeof(double));
    delete S->pool;  // returns every cached block
    destroy_streams(S);
    delete S;
}
