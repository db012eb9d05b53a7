// Launcher of the entropic step with per-site start values of its search
// (defined in entropic.hpp, instantiated in kernels_<storage>_ent.hip).
#pragma once

#include "types.hpp"

namespace lbm81 {

// warm: one float per site (site order [sub][z][y][x]) read as the start of
// the search for alpha and overwritten with the alpha found (negative where
// positivity capped it); nullptr for none.
template <int ST>
void launch_step_entropic_warm(void *f, const Geom &g, double omega,
                               unsigned *flags, bool odd, float *warm,
                               hipStream_t stream);

}  // namespace lbm81
