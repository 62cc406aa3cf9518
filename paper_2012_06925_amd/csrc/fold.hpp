// fold.hpp -- layout shared by the host packer and the device passes for the
// deterministic symmetric passes (plain structs, no HIP types).
//
// A symmetric pass evaluates each pair once for both sides.  Instead of adding
// to the outputs with atomics (whose order varies run to run), item i writes
// its target sums to slots[ibase[i] + r] (r < the item's target count) and
// then the partial sums of its sources, entry after entry.  A fold pass adds
// to every output, in a fixed order, the slot values that belong to it:
// segment s covers outputs [0, n) at `off` of phi (deg < 0) or of the proxy
// potentials of degree deg, and its parts pb .. pe-1 each give the values
// slots[slot + k - lo] of its outputs k in [lo, lo + len).  (In a batch the
// PC/CP items, whose targets are particles and whose sources are proxies,
// write their target sums to the particle fold's slots and their source
// partials to the proxy fold's; each fold then takes parts from two item
// lists, FoldGroup in engine.hpp.)
#pragma once

#include <cstdint>

namespace bldtt {

struct FoldPart {
    int64_t slot;
    int32_t lo, len;
};

struct FoldSeg {
    int64_t off;
    int32_t n, deg;
    int32_t pb, pe;
};

}  // namespace bldtt
