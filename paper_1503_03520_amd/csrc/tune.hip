// Autotuner cache (tune.hpp) and its C entry points.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "common.hpp"
#include "tune.hpp"

namespace {

std::mutex g_mu;
std::map<std::string, int> g_choice;
bool g_loaded = false;

const char* cache_path() { return std::getenv("L1LS_TUNE_CACHE"); }

// {"l1ls_tune": 1, "choices": {"key": 3, ...}}: keys hold no quotes or
// backslashes, values are small integers.
void load_locked() {
    g_loaded = true;
    const char* path = cache_path();
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "rb");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, k);
    std::fclose(f);
    const size_t c = text.find("\"choices\"");
    if (c == std::string::npos) return;
    size_t p = text.find('{', c);
    while (p != std::string::npos) {
        const size_t q0 = text.find('"', p + 1);
        const size_t end = text.find('}', p + 1);
        if (q0 == std::string::npos || (end != std::string::npos && end < q0)) break;
        const size_t q1 = text.find('"', q0 + 1);
        const size_t colon = text.find(':', q1);
        if (q1 == std::string::npos || colon == std::string::npos) break;
        const int v = std::atoi(text.c_str() + colon + 1);
        const std::string key = text.substr(q0 + 1, q1 - q0 - 1);
        if (g_choice.find(key) == g_choice.end()) g_choice[key] = v;
        p = text.find(',', colon);
    }
}

void save_locked() {
    const char* path = cache_path();
    if (!path || !*path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    std::fprintf(f, "{\"l1ls_tune\": 1, \"choices\": {");
    bool first = true;
    for (const auto& kv : g_choice) {
        std::fprintf(f, "%s\n  \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
        first = false;
    }
    std::fprintf(f, "\n}}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

}  // namespace

int tune_lookup(const std::string& key) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_loaded) load_locked();
    auto it = g_choice.find(key);
    return it == g_choice.end() ? -1 : it->second;
}

void tune_store(const std::string& key, int choice) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_loaded) load_locked();
    if (choice < 0)
        g_choice.erase(key);
    else
        g_choice[key] = choice;
    save_locked();
}

int tune_size_class(int64_t rows) {
    int c = 0;
    while (((int64_t)1 << c) < rows) ++c;
    return c;
}

extern "C" int32_t l1ls_tune_get(const char* key) { return key ? tune_lookup(key) : -1; }

extern "C" l1ls_status l1ls_tune_set(const char* key, int32_t choice) {
    if (!key || !*key) return L1LS_E_ARG;
    for (const char* c = key; *c; ++c)
        if (*c == '"' || *c == '\\' || *c == '\n') return L1LS_E_ARG;
    tune_store(key, choice);
    return L1LS_OK;
}
