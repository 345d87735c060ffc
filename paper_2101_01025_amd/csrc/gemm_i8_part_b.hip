// Instantiations of the grouped INT8 product kernel for the configurations of
// list B (gemm_i8_configs.h).
#include "gemm_i8_kernel.h"

namespace ffa {
FFA_I8_PART(b, FFA_I8_CONFIGS_B)
}  // namespace ffa
