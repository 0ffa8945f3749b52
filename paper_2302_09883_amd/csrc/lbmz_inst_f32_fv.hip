// Kernel instantiations: float, scheme S_FV (upwind transport), patch sizes [8, 16, 32, 64], Haar and BL5/3, float32 records.
#include "lbmz_patch_kernel.h"

namespace lbmz {

bool dispatch_f32_fv(LBMZ_DISPATCH_ARGS) {
  if (k.dtype != 0 || k.scheme != S_FV) return false;
  LBMZ_CASE_T(float, 8, W_HAAR, S_FV, VF_F32)
  LBMZ_CASE_T(float, 8, W_BL53, S_FV, VF_F32)
  LBMZ_CASE_T(float, 16, W_HAAR, S_FV, VF_F32)
  LBMZ_CASE_T(float, 16, W_BL53, S_FV, VF_F32)
  LBMZ_CASE_T(float, 32, W_HAAR, S_FV, VF_F32)
  LBMZ_CASE_T(float, 32, W_BL53, S_FV, VF_F32)
  LBMZ_CASE_T(float, 64, W_HAAR, S_FV, VF_F32)
  LBMZ_CASE_T(float, 64, W_BL53, S_FV, VF_F32)
  return false;
}

}  // namespace lbmz
