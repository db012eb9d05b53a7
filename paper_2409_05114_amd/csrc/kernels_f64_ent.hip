// Entropic-collision step kernels of the F64 storage form (see
// entropic.hpp), compiled on their own.
#include "entropic.hpp"

template void lbm81::launch_step_entropic<LBM_F64>(
    void *, const lbm81::Geom &, double, unsigned *, bool, hipStream_t);
template void lbm81::launch_step_entropic_warm<LBM_F64>(
    void *, const lbm81::Geom &, double, unsigned *, bool, float *,
    hipStream_t);
