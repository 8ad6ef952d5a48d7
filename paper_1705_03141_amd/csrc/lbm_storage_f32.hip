// lbm_storage_f32.hip -- kernels instantiated for float population storage.
#include "lbm_step.h"

namespace lbm {
LBM_INSTANTIATE_STORAGE(float)
LBM_INSTANTIATE_STEP(float)
}  // namespace lbm
