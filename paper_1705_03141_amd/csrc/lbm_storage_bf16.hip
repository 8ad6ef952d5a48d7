// lbm_storage_bf16.hip -- kernels instantiated for bf16 population storage.
#include "lbm_step.h"

namespace lbm {
LBM_INSTANTIATE_STORAGE(bf16)
LBM_INSTANTIATE_STEP(bf16)
}  // namespace lbm
