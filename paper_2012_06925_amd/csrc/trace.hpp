// trace.hpp -- named host ranges (roctx) around the library's host phases:
// setup, compute, traversal, degree choice, and the launches of each GPU
// phase.  `rocprofv3 --marker-trace` shows them on the host timeline beside
// the kernels; without a profiler attached the calls return at once.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace bldtt {

struct HostRange {
    explicit HostRange(const char* name) { roctxRangePushA(name); }
    ~HostRange() { roctxRangePop(); }
    HostRange(const HostRange&) = delete;
    HostRange& operator=(const HostRange&) = delete;
};

// Range names of the GPU phases (BLDTT_PH_* order).
inline const char* phase_range_name(int ph) {
    static const char* const names[] = {"bldtt:launch up",        "bldtt:launch cp_cc",   "bldtt:launch down_transfer",
                                        "bldtt:launch pp_pc",     "bldtt:launch down_leaf", "bldtt:launch pp_pc_sep",
                                        "bldtt:launch pp_sym",    "bldtt:launch pp_self"};
    return ph >= 0 && ph < 8 ? names[ph] : "bldtt:launch";
}

}  // namespace bldtt
