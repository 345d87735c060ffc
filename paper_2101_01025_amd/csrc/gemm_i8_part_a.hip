// Instantiations of the grouped INT8 product kernel for the configurations of
// list A (gemm_i8_configs.h).
#include "gemm_i8_kernel.h"

namespace ffa {
FFA_I8_PART(a, FFA_I8_CONFIGS_A)
}  // namespace ffa
