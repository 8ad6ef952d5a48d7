// lbm_storage_f32.hip -- kernels instantiated for float population storage.
#include "lbm_kernels_impl.h"

namespace lbm {
LBM_INSTANTIATE_STORAGE(float)
}  // namespace lbm
