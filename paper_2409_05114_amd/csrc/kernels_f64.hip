// Kernels of the F64 storage form (see kernels.hpp); the entropic and
// series step kernels are in kernels_f64_ent.hip and kernels_f64_ser.hip.
#include "kernels.hpp"

extern template void lbm81::launch_step_entropic<LBM_F64>(
    void *, const lbm81::Geom &, double, unsigned *, bool, hipStream_t);
extern template void lbm81::launch_step_series<LBM_F64>(
    void *, const lbm81::Geom &, double, unsigned *, bool, hipStream_t);
template struct lbm81::Launch<LBM_F64>;
