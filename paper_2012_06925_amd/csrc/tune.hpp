// tune.hpp -- the tile autotuner's cache: choices keyed by a short string,
// held in memory and mirrored in an optional text file.
#pragma once

#include <cstdint>
#include <string>

namespace bldtt {

struct TuneChoice {
    int tpt = 2;              // targets per thread, particle items
    int tpt_proxy = 2;        // targets per thread, proxy items
    int groups_per_cu = 0;    // resident work groups per CU (batch kernel; 0 = as many as fit)
    double ms = 0.0;          // measured device time of the choice
};

// Key: kind, precision, degree mode, leaf size and ceil(log2(size)).
std::string tune_key(const char* what, int kind, bool fp32, bool varied, int degree, int64_t leaf, int64_t size,
                     int64_t count);

void tune_set_path(const char* path);
bool tune_lookup(const std::string& key, TuneChoice& out);
void tune_store(const std::string& key, const TuneChoice& c);

}  // namespace bldtt
