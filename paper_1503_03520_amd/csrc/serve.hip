// Serving scheduler: continuous batching of l1-LS solve requests on one GPU.
//
// Requests (instance parameters of Procedure IGen, section 3.1, and a
// relative-gap tolerance) wait in a FIFO queue.  Each tick:
//  1. admission: while the head of the queue fits the HBM budget (its
//     footprint estimated before generation from the bound of 4^rounds
//     nonzeros per column of A = Q Sigma G^T, eq. (16)) and a batch slot is
//     free, generate its instance on the device and add it to the batch;
//  2. run `iters_per_tick` FISTA iterations of every resident slot (one
//     shared launch per pass, see batch.hip);
//  3. retire the slots whose gap test passed (or hit their iteration cap):
//     copy the iterate to a result buffer, free the slot and the instance.
// Iterates stay on the device from admission to retirement.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <unordered_map>
#include <vector>

#include "common.hpp"

using ServeClock = std::chrono::steady_clock;

struct ServeReq {
    int64_t id;
    l1ls_request r;
    ServeClock::time_point submitted;
};

struct ServeSlot {
    int64_t id = -1;
    l1ls_instance* inst = nullptr;
    int64_t max_iter = 0;
    ServeClock::time_point submitted;
};

struct ServeDone {
    double* x = nullptr;  // n FP64 on the device
    int64_t n = 0;
    l1ls_report rep;
};

struct l1ls_server {
    int32_t max_slots = 0, iters_per_tick = 0;
    size_t budget = 0, used = 0;
    hipStream_t stream = nullptr;
    l1ls_batch* batch = nullptr;
    int64_t next_id = 0;
    std::deque<ServeReq> queue;
    std::vector<ServeSlot> slots;
    std::vector<size_t> est;
    std::unordered_map<int64_t, ServeDone> done;
    std::vector<int64_t> fresh;  // completed since the last l1ls_server_completed call
    int64_t ticks = 0;
};

size_t batch_slot_bytes(int64_t m, int64_t n);

namespace {

// The terms of l1ls_instance_footprint for an FP32-only instance, with nnz
// at its bound (each Givens stage at most doubles a column's support).
size_t estimate_footprint(const l1ls_request& r) {
    const size_t nnz = (size_t)r.n * (r.rounds >= 2 ? 16 : 4);
    return nnz * 16 + (size_t)(r.m + r.n + 2) * 4 + (size_t)(r.m + r.n) * 48 + batch_slot_bytes(r.m, r.n);
}

bool valid_request(const l1ls_request& r) {
    return r.n >= 2 && r.m >= r.n && r.m % 2 == 0 && r.n % 2 == 0 && r.s >= 0 && r.s <= r.n && r.kappa >= 1.0 &&
           r.tau > 0.0 && (r.rounds == 1 || r.rounds == 2) && r.rel_gap_tol > 0.0 && r.max_iter > 0;
}

}  // namespace

extern "C" l1ls_status l1ls_server_create(int32_t max_slots, size_t hbm_budget_bytes, int32_t iters_per_tick,
                                          int32_t check_every, void* stream, l1ls_server** out) {
    if (!out || max_slots < 1 || iters_per_tick < 1 || check_every < 1) return L1LS_E_ARG;
    *out = nullptr;
    l1ls_solve_opts o;
    l1ls_solve_opts_default(&o);
    o.precision = L1LS_F32;
    o.op = L1LS_OP_STORED;
    o.check_every = check_every;
    o.rel_gap_tol = 1e-6;  // per slot tolerances are set at admission
    o.stream = stream;
    l1ls_server* S = new l1ls_server();
    S->max_slots = max_slots;
    S->iters_per_tick = iters_per_tick;
    S->budget = hbm_budget_bytes;
    S->stream = (hipStream_t)stream;
    S->slots.assign(max_slots, ServeSlot{});
    S->est.assign(max_slots, 0);
    l1ls_status st = l1ls_batch_create(max_slots, 0, &o, &S->batch);
    if (st != L1LS_OK) {
        delete S;
        return st;
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
    S->queue.push_back(q);
    *id_out = q.id;
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_server_tick(l1ls_server* S, int32_t* admitted, int32_t* completed) {
    if (!S) return L1LS_E_ARG;
    int32_t na = 0, nc = 0;
    // 1. admission (FIFO, by footprint and free slots)
    while (!S->queue.empty()) {
        const l1ls_request& r = S->queue.front().r;
        const size_t fp = estimate_footprint(r);
        if (S->budget && S->used + fp > S->budget) break;
        int slot = -1;
        for (int q = 0; q < S->max_slots; ++q)
            if (S->slots[q].id < 0) {
                slot = q;
                break;
            }
        if (slot < 0) break;
        l1ls_gen_opts go;
        go.rounds = r.rounds;
        go.storage = L1LS_STORE_F32;
        go.stream = S->stream;
        go.layout = L1LS_LAYOUT_STAGE;
        l1ls_instance* inst = nullptr;
        L1LS_TRY(l1ls_generate_ex(r.m, r.n, r.kappa, r.s, r.tau, r.seed, &go, &inst));
        int32_t bslot = -1;
        l1ls_status st = l1ls_batch_add_ex(S->batch, inst, r.tau, r.rel_gap_tol, r.max_iter, &bslot);
        if (st != L1LS_OK) {
            l1ls_free(inst);
            return st;
        }
        S->slots[bslot].id = S->queue.front().id;
        S->slots[bslot].inst = inst;
        S->slots[bslot].max_iter = r.max_iter;
        S->slots[bslot].submitted = S->queue.front().submitted;
        S->est[bslot] = fp;
        S->used += fp;
        S->queue.pop_front();
        ++na;
    }
    // 2. iterations of the resident set
    L1LS_TRY(l1ls_batch_iterate(S->batch, S->iters_per_tick));
    ++S->ticks;
    // 3. retirement
    std::vector<l1ls_report> reps(S->max_slots);
    L1LS_TRY(l1ls_batch_poll(S->batch, reps.data(), nullptr));
    for (int q = 0; q < S->max_slots; ++q) {
        ServeSlot& sl = S->slots[q];
        if (sl.id < 0) continue;
        const l1ls_report& rp = reps[q];
        if (rp.converged == 0 && rp.iterations < sl.max_iter) continue;  // still iterating
        ServeDone d;
        d.n = sl.inst->n;
        d.rep = rp;
        d.rep.seconds = std::chrono::duration<double>(ServeClock::now() - sl.submitted).count();
        void* p = nullptr;
        HIP_TRY(hipMalloc(&p, d.n * sizeof(double)));
        d.x = (double*)p;
        L1LS_TRY(l1ls_batch_get_x(S->batch, q, d.x));
        L1LS_TRY(l1ls_batch_remove(S->batch, q));
        l1ls_free(sl.inst);
        S->used -= S->est[q];
        S->est[q] = 0;
        S->done[sl.id] = d;
        S->fresh.push_back(sl.id);
        sl = ServeSlot{};
        ++nc;
    }
    if (admitted) *admitted = na;
    if (completed) *completed = nc;
    return L1LS_OK;
}

extern "C" int32_t l1ls_server_completed(l1ls_server* S, int64_t* ids, int32_t cap) {
    if (!S || !ids || cap < 1) return 0;
    const int32_t k = (int32_t)std::min<size_t>((size_t)cap, S->fresh.size());
    for (int32_t q = 0; q < k; ++q) ids[q] = S->fresh[q];
    S->fresh.erase(S->fresh.begin(), S->fresh.begin() + k);
    return k;
}

extern "C" l1ls_status l1ls_server_take(l1ls_server* S, int64_t id, double* x_out_dev, l1ls_report* rep) {
    if (!S) return L1LS_E_ARG;
    auto it = S->done.find(id);
    if (it == S->done.end()) return L1LS_E_STATE;
    if (x_out_dev)
        HIP_TRY(hipMemcpyAsync(x_out_dev, it->second.x, it->second.n * sizeof(double), hipMemcpyDeviceToDevice,
                               S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
    if (rep) *rep = it->second.rep;
    (void)hipFree(it->second.x);
    S->done.erase(it);
    return L1LS_OK;
}

extern "C" l1ls_status l1ls_server_stats(l1ls_server* S, int32_t* queued, int32_t* resident, size_t* used_bytes) {
    if (!S) return L1LS_E_ARG;
    int32_t res = 0;
    for (const ServeSlot& s : S->slots) res += (s.id >= 0);
    if (queued) *queued = (int32_t)S->queue.size();
    if (resident) *resident = res;
    if (used_bytes) *used_bytes = S->used;
    return L1LS_OK;
}

extern "C" size_t l1ls_request_footprint(const l1ls_request* r) {
    return (r && valid_request(*r)) ? estimate_footprint(*r) : 0;
}

extern "C" void l1ls_server_destroy(l1ls_server* S) {
    if (!S) return;
    (void)hipStreamSynchronize(S->stream);
    for (ServeSlot& s : S->slots)
        if (s.inst) l1ls_free(s.inst);
    for (auto& kv : S->done) (void)hipFree(kv.second.x);
    l1ls_batch_destroy(S->batch);
    delete S;
}
