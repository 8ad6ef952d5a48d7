// lbm_dispatch.hip -- storage-type dispatch of the kernel launchers.
#include "lbm_kernels.h"

namespace lbm {

bool step_tiling_supported(int tx, int ty) {
  return (tx == 32 && (ty == 4 || ty == 8 || ty == 16)) || (tx == 64 && (ty == 4 || ty == 8));
}


hipError_t launch_step(int storage, const StepArgs& a, int tx, int ty, hipStream_t s) {
  switch (storage) {
    case 0: return launch_step_T<float>(a, tx, ty, s);
    case 1: return launch_step_T<_Float16>(a, tx, ty, s);
    case 2: return launch_step_T<bf16>(a, tx, ty, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch(int storage, const StepArgs* cases, const int* first, int ncases, int nblocks, bool init,
                        int tx, int ty, int lat, hipStream_t s) {
  switch (storage) {
    case 0: return launch_batch_T<float>(cases, first, ncases, nblocks, init, tx, ty, lat, s);
    case 1: return launch_batch_T<_Float16>(cases, first, ncases, nblocks, init, tx, ty, lat, s);
    case 2: return launch_batch_T<bf16>(cases, first, ncases, nblocks, init, tx, ty, lat, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_inflow(int storage, const StepArgs& a, hipStream_t s) {
  switch (storage) {
    case 0: return launch_inflow_T<float>(a, s);
    case 1: return launch_inflow_T<_Float16>(a, s);
    case 2: return launch_inflow_T<bf16>(a, s);
  }
  return hipErrorInvalidValue;
}

int step_resident_blocks(int storage, int tx, int ty, int device) {
  switch (storage) {
    case 0: return step_resident_blocks_T<float>(tx, ty, device);
    case 1: return step_resident_blocks_T<_Float16>(tx, ty, device);
    case 2: return step_resident_blocks_T<bf16>(tx, ty, device);
  }
  return 0;
}

hipError_t launch_outlet(int storage, const AuxArgs& a, hipStream_t s) {
  switch (storage) {
    case 0: return launch_outlet_T<float>(a, s);
    case 1: return launch_outlet_T<_Float16>(a, s);
    case 2: return launch_outlet_T<bf16>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_outlet(int storage, const AuxArgs* cases, const int* first, int ncases, int nblocks,
                               long long step, hipStream_t s) {
  switch (storage) {
    case 0: return launch_batch_outlet_T<float>(cases, first, ncases, nblocks, step, s);
    case 1: return launch_batch_outlet_T<_Float16>(cases, first, ncases, nblocks, step, s);
    case 2: return launch_batch_outlet_T<bf16>(cases, first, ncases, nblocks, step, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_inflow(int storage, const StepArgs* cases, const int* first, int ncases, int nblocks,
                               long long step, hipStream_t s) {
  switch (storage) {
    case 0: return launch_batch_inflow_T<float>(cases, first, ncases, nblocks, step, s);
    case 1: return launch_batch_inflow_T<_Float16>(cases, first, ncases, nblocks, step, s);
    case 2: return launch_batch_inflow_T<bf16>(cases, first, ncases, nblocks, step, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fields(int storage, const AuxArgs& a, int x0, int y0, int z0, int wx, int wy, int wz, double* out,
                         hipStream_t s) {
  switch (storage) {
    case 0: return launch_fields_T<float>(a, x0, y0, z0, wx, wy, wz, out, s);
    case 1: return launch_fields_T<_Float16>(a, x0, y0, z0, wx, wy, wz, out, s);
    case 2: return launch_fields_T<bf16>(a, x0, y0, z0, wx, wy, wz, out, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_populations(int storage, const AuxArgs& a, double* out, hipStream_t s) {
  switch (storage) {
    case 0: return launch_populations_T<float>(a, out, s);
    case 1: return launch_populations_T<_Float16>(a, out, s);
    case 2: return launch_populations_T<bf16>(a, out, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_coarse(int storage, const AuxArgs& a, int f, float inv_u, float* out, int ph, int pw, hipStream_t s) {
  switch (storage) {
    case 0: return launch_coarse_T<float>(a, f, inv_u, out, ph, pw, s);
    case 1: return launch_coarse_T<_Float16>(a, f, inv_u, out, ph, pw, s);
    case 2: return launch_coarse_T<bf16>(a, f, inv_u, out, ph, pw, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_diag(int storage, const AuxArgs& a, const DiagQuery& q, double* part, long long nblocks,
                       double* out, hipStream_t s) {
  switch (storage) {
    case 0: return launch_diag_T<float>(a, q, part, nblocks, out, s);
    case 1: return launch_diag_T<_Float16>(a, q, part, nblocks, out, s);
    case 2: return launch_diag_T<bf16>(a, q, part, nblocks, out, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
