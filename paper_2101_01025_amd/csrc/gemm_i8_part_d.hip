// Instantiations of the grouped INT8 product kernel for the configurations of
// list D (gemm_i8_configs.h).
#include "gemm_i8_kernel.h"

namespace ffa {
FFA_I8_PART(d, FFA_I8_CONFIGS_D)
}  // namespace ffa
