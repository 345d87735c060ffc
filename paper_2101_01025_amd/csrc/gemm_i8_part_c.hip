// Instantiations of the grouped INT8 product kernel for the configurations of
// list C (gemm_i8_configs.h).
#include "gemm_i8_kernel.h"

namespace ffa {
FFA_I8_PART(c, FFA_I8_CONFIGS_C)
}  // namespace ffa
