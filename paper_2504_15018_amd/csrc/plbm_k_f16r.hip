// Kernels for population storage StF16R (half, per-node reference shift).
#define PLBM_ST plbm::StF16R
#define PLBM_SUFFIX f16r
#include "plbm_kernels_inst.hpp"
