// Placement probe launcher (placement.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "types.hpp"

namespace lbm81 {

// Enqueue one pass of the probe over the populations at f (layout of
// `storage` for geometry g) on `stream`; false for an unknown storage.
bool launch_placement(void *f, const Geom &g, int storage, hipStream_t stream);

}  // namespace lbm81
