// Autotuning cache: tuned launch parameters per size class, kept for the
// process and optionally in a text file named by S7_TUNE_CACHE (one class per
// line: "s7tune1 kind tag unit nbucket sbucket v0 v1").  The timing trials
// themselves live beside the kernels they launch (s7_single.hip).
#include <cstdlib>
#include <map>
#include <mutex>

#include "s7_host.hpp"

namespace s7 {

bool TuneKey::operator<(const TuneKey& o) const {
    if (kind != o.kind) return kind < o.kind;
    if (tag != o.tag) return tag < o.tag;
    if (unit != o.unit) return unit < o.unit;
    if (nbucket != o.nbucket) return nbucket < o.nbucket;
    return sbucket < o.sbucket;
}

namespace {

std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;
bool g_tune_loaded = false;

const char* cache_path() {
    const char* p = std::getenv("S7_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

void load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = cache_path();
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char tag[16];
    TuneKey k;
    int v0, v1;
    while (std::fscanf(f, "%15s %d %d %d %d %d %d %d", tag, &k.kind, &k.tag, &k.unit, &k.nbucket,
                       &k.sbucket, &v0, &v1) == 8) {
        if (std::string(tag) == "s7tune1") g_tune[k] = {v0, v1};
    }
    std::fclose(f);
}

}  // namespace

bool tune_lookup(const TuneKey& k, int (&val)[2]) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_locked();
    auto it = g_tune.find(k);
    if (it == g_tune.end()) return false;
    val[0] = it->second.first;
    val[1] = it->second.second;
    return true;
}

void tune_store(const TuneKey& k, const int (&val)[2]) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_locked();
    g_tune[k] = {val[0], val[1]};
    const char* path = cache_path();
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;  // an unwritable cache file only costs re-tuning in later processes
    std::fprintf(f, "s7tune1 %d %d %d %d %d %d %d\n", k.kind, k.tag, k.unit, k.nbucket, k.sbucket,
                 val[0], val[1]);
    std::fclose(f);
}

}  // namespace s7
