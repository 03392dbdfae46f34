// Kernels for population storage StF32.
#define PLBM_ST plbm::StF32
#define PLBM_SUFFIX f32
#include "plbm_kernels_inst.hpp"
