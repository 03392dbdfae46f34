// Kernels for population storage StBF16S.
#define PLBM_ST plbm::StBF16S
#define PLBM_SUFFIX bf16s
#include "plbm_kernels_inst.hpp"
