// Static device scratch of the allocation-free product (scratch.hip).
#pragma once

#include <cstddef>

namespace dh2 {

// Size of the static scratch array (per GPU): the largest staging arena of a
// handle's product (gathered X, its row-major copy, Y in cluster order and
// the slot vectors, for max_nrhs right-hand sides) that dh2_matvec_noalloc
// accepts.
constexpr size_t kScratchBytes = (size_t)64 << 20;

// Device address of the current device's copy of the array, looked up once
// per device (hipGetSymbolAddress) and kept; nullptr if the lookup failed.
// *bytes (may be NULL) receives kScratchBytes.
void* scratch_region(size_t* bytes);

}  // namespace dh2
