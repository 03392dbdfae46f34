// Kernels for population storage StF16S.
#define PLBM_ST plbm::StF16S
#define PLBM_SUFFIX f16s
#include "plbm_kernels_inst.hpp"
