// Kernels for population storage StBF16R (bfloat16, per-node reference shift).
#define PLBM_ST plbm::StBF16R
#define PLBM_SUFFIX bf16r
#include "plbm_kernels_inst.hpp"
