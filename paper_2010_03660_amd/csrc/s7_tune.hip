// Autotuning cache: tuned launch parameters per size class, kept for the
// process and optionally in a text file named by S7_TUNE_CACHE (one class per
// line: "s7tune2 kind tag unit nbucket sbucket v0 v1 v2 v3"; lines of the
// older two-value form read with v2 = v3 = 0).  The timing trials themselves
// live beside the kernels they launch (s7_single.hip); S7_TUNE_LOG names a
// file that receives one line per trial.
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
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
std::map<TuneKey, std::array<int, 4>> g_tune;
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
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        char tag[16];
        TuneKey k;
        int v[4] = {0, 0, 0, 0};
        const int got = std::sscanf(line, "%15s %d %d %d %d %d %d %d %d %d", tag, &k.kind, &k.tag, &k.unit,
                                    &k.nbucket, &k.sbucket, &v[0], &v[1], &v[2], &v[3]);
        if ((std::strcmp(tag, "s7tune1") == 0 && got >= 8) || (std::strcmp(tag, "s7tune2") == 0 && got == 10))
            g_tune[k] = {v[0], v[1], v[2], v[3]};
    }
    std::fclose(f);
}

}  // namespace

bool tune_lookup(const TuneKey& k, int (&val)[4]) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_locked();
    auto it = g_tune.find(k);
    if (it == g_tune.end()) return false;
    for (int i = 0; i < 4; ++i) val[i] = it->second[i];
    return true;
}

void tune_store(const TuneKey& k, const int (&val)[4]) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_locked();
    g_tune[k] = {val[0], val[1], val[2], val[3]};
    const char* path = cache_path();
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;  // an unwritable cache file only costs re-tuning in later processes
    std::fprintf(f, "s7tune2 %d %d %d %d %d %d %d %d %d\n", k.kind, k.tag, k.unit, k.nbucket, k.sbucket,
                 val[0], val[1], val[2], val[3]);
    std::fclose(f);
}

void tune_log(const char* line) {
    const char* p = std::getenv("S7_TUNE_LOG");
    if (!p || !*p) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE* f = std::fopen(p, "a");
    if (!f) return;
    std::fprintf(f, "%s\n", line);
    std::fclose(f);
}

}  // namespace s7
