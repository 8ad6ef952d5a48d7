// lbm_storage_f16.hip -- kernels instantiated for _Float16 population storage.
#include "lbm_step.h"

namespace lbm {
LBM_INSTANTIATE_STORAGE(_Float16)
LBM_INSTANTIATE_STEP(_Float16)
}  // namespace lbm
