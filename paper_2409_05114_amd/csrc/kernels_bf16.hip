// Kernels of the BF16 storage form (see kernels.hpp).
#include "kernels.hpp"

template struct lbm81::Launch<LBM_BF16>;
