// Series-equilibrium step kernels of the BF16 storage form (see
// kernels.hpp), compiled on their own.
#include "kernels.hpp"

template void lbm81::launch_step_series<LBM_BF16>(
    void *, const lbm81::Geom &, double, unsigned *, bool, hipStream_t);
