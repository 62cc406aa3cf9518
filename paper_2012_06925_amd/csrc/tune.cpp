// tune.cpp -- autotune cache (see tune.hpp and bldtt_set_tune_cache).
#include "tune.hpp"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>

namespace bldtt {
namespace {

struct Cache {
    std::mutex m;
    std::string path;          // "" = memory only
    bool path_set = false;     // set by tune_set_path (else the environment decides)
    bool loaded = false;
    std::map<std::string, TuneChoice> entries;
};

Cache& cache() {
    static Cache c;
    return c;
}

std::string current_path(Cache& c) {
    if (c.path_set) return c.path;
    const char* e = std::getenv("BLDTT_TUNE_CACHE");
    return e ? std::string(e) : std::string();
}

void load(Cache& c) {
    if (c.loaded) return;
    c.loaded = true;
    std::string p = current_path(c);
    if (p.empty()) return;
    std::ifstream f(p);
    std::string line;
    while (std::getline(f, line)) {
        size_t tab = line.find('\t');
        if (tab == std::string::npos) continue;
        TuneChoice t;
        std::istringstream rest(line.substr(tab + 1));
        if (rest >> t.tpt >> t.tpt_proxy >> t.groups_per_cu >> t.ms) c.entries[line.substr(0, tab)] = t;
    }
}

void save(Cache& c) {
    std::string p = current_path(c);
    if (p.empty()) return;
    std::string tmp = p + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return;                        // an unwritable cache is not an error
        for (const auto& kv : c.entries)
            f << kv.first << '\t' << kv.second.tpt << ' ' << kv.second.tpt_proxy << ' ' << kv.second.groups_per_cu
              << ' ' << kv.second.ms << '\n';
    }
    std::rename(tmp.c_str(), p.c_str());
}

}  // namespace

std::string tune_key(const char* what, int kind, bool fp32, bool varied, int degree, int64_t leaf, int64_t size,
                     int64_t count) {
    int lg = 0;
    while ((int64_t(1) << lg) < size && lg < 62) ++lg;
    std::ostringstream k;
    k << what << ":kind=" << kind << ":fp32=" << (fp32 ? 1 : 0) << ":varied=" << (varied ? 1 : 0)
      << ":degree=" << degree << ":leaf=" << leaf << ":log2n=" << lg << ":count=" << count;
    return k.str();
}

void tune_set_path(const char* path) {
    Cache& c = cache();
    std::lock_guard<std::mutex> g(c.m);
    c.path_set = path != nullptr;
    c.path = path ? path : "";
    c.loaded = false;
    c.entries.clear();
}

bool tune_lookup(const std::string& key, TuneChoice& out) {
    Cache& c = cache();
    std::lock_guard<std::mutex> g(c.m);
    load(c);
    auto it = c.entries.find(key);
    if (it == c.entries.end()) return false;
    out = it->second;
    return true;
}

void tune_store(const std::string& key, const TuneChoice& t) {
    Cache& c = cache();
    std::lock_guard<std::mutex> g(c.m);
    load(c);
    c.entries[key] = t;
    save(c);
}

}  // namespace bldtt
