// Autotuner cache: the factorisation's schedule settings (panels per
// trailing-update group, cap on the group update's workgroups) chosen per
// (device architecture, HIP runtime, precision, order rounded to a power of
// two), and the batched solver's persistent grid per batch size.  Kept in
// memory for the process and, when SPD_TUNE_CACHE names a file, persisted
// there as a small JSON object (one entry per line, rewritten whole on every
// store).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "internal.h"

namespace spd {
namespace {

std::mutex g_mu;
bool g_loaded = false;
std::map<std::string, TuneVal> g_tab;

const char *cache_path() { return std::getenv("SPD_TUNE_CACHE"); }

std::string device_tag()
{
    int dev = 0, ver = 0;
    hipDeviceProp_t p;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) {
        arch = p.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch.resize(colon);
    }
    (void)hipRuntimeGetVersion(&ver);
    return arch + "|hip" + std::to_string(ver);
}

// the entries this file format writes: "key": {"a": 1, "b": 2, "c": 3, "ms": 4.5}
void load_locked()
{
    g_loaded = true;
    const char *path = cache_path();
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        const char *q0 = std::strchr(line, '"');
        const char *q1 = q0 ? std::strchr(q0 + 1, '"') : nullptr;
        if (!q0 || !q1) continue;
        const std::string key(q0 + 1, q1);
        TuneVal v;
        const char *b = std::strchr(q1, '{');
        if (!b || std::sscanf(b, "{\"a\": %d, \"b\": %d, \"c\": %d, \"ms\": %lf}", &v.a, &v.b, &v.c, &v.ms) != 4)
            continue;
        g_tab[key] = v;
    }
    std::fclose(f);
}

void save_locked()
{
    const char *path = cache_path();
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : g_tab) {
        std::fprintf(f, "  \"%s\": {\"a\": %d, \"b\": %d, \"c\": %d, \"ms\": %.6f}%s\n", kv.first.c_str(), kv.second.a,
                     kv.second.b, kv.second.c, kv.second.ms, (++i < g_tab.size()) ? "," : "");
    }
    std::fprintf(f, "}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

}  // namespace

int64_t tune_bucket(int64_t n)
{
    if (n <= 1) return 1;
    const int k = (int)std::lround(std::log2((double)n));
    return (int64_t)1 << k;
}

std::string tune_key(const char *kind, int64_t size) { return device_tag() + "|" + kind + "|" + std::to_string(size); }

int tune_lookup(const std::string &key, TuneVal *v)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_loaded) {
        load_locked();
        if (g_tab.count(key)) {
            *v = g_tab[key];
            return 2;  // from the file
        }
    }
    auto it = g_tab.find(key);
    if (it == g_tab.end()) return 0;
    *v = it->second;
    return 1;
}

void tune_store(const std::string &key, const TuneVal &v)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_loaded) load_locked();
    g_tab[key] = v;
    save_locked();
}

void tune_clear()
{
    std::lock_guard<std::mutex> g(g_mu);
    g_tab.clear();
    g_loaded = false;  // the next lookup reads the file again
}

}  // namespace spd
