// The library's device-memory source (l1ls_set_allocator): every block the
// library allocates outside a caller-given pool comes from the installed
// allocator, else from hipMalloc.  A block goes back to the allocator that
// made it, even when another one has been installed since.
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace {

struct Source {
    l1ls_allocator a;
};

std::mutex g_mu;
const Source* g_current = nullptr;            // nullptr: hipMalloc / hipFree
std::vector<const Source*> g_sources;         // every installed allocator (kept for their blocks)
std::unordered_map<void*, const Source*> g_owner;  // blocks made by an installed allocator

}  // namespace

l1ls_status lib_alloc(void** p, size_t bytes) {
    *p = nullptr;
    const Source* src;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        src = g_current;
    }
    if (!src) {
        const hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? L1LS_E_NOMEM : L1LS_E_HIP;
        return L1LS_OK;
    }
    void* q = src->a.alloc(src->a.ctx, bytes);
    if (!q) return L1LS_E_NOMEM;
    std::lock_guard<std::mutex> lk(g_mu);
    g_owner[q] = src;
    *p = q;
    return L1LS_OK;
}

void lib_free(void* p, size_t bytes, bool synced) {
    if (!p) return;
    const Source* src = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_owner.find(p);
        if (it != g_owner.end()) {
            src = it->second;
            g_owner.erase(it);
        }
    }
    if (!src) {
        (void)hipFree(p);
        return;
    }
    // hipFree waits for the device before it releases a block; a caller's
    // allocator may hand the block to another stream at once, so wait here
    // (unless the caller just did)
    if (!synced) (void)hipDeviceSynchronize();
    src->a.free(src->a.ctx, p, bytes);
}

extern "C" l1ls_status l1ls_set_allocator(const l1ls_allocator* a) {
    if (a && (!a->alloc || !a->free)) return L1LS_E_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!a) {
        g_current = nullptr;
        return L1LS_OK;
    }
    Source* s = new Source{*a};
    g_sources.push_back(s);
    g_current = s;
    return L1LS_OK;
}

extern "C" size_t l1ls_instance_bytes(const l1ls_instance* inst) {
    if (!inst) return 0;
    size_t total = 0;
    for (const auto& pr : inst->arena.ptrs) total += pr.second;
    return total;
}
