// Kernels of the F32 storage form (see kernels.hpp).
#include "kernels.hpp"

template struct lbm81::Launch<LBM_F32>;
