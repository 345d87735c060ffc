// Instantiations of the grouped INT8 product kernel for the configurations of
// list E (gemm_i8_configs.h).
#include "gemm_i8_kernel.h"

namespace ffa {
FFA_I8_PART(e, FFA_I8_CONFIGS_E)
}  // namespace ffa
