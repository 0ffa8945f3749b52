// Kernel instantiations: float, scheme S_EULER (compressible Euler, Rusanov flux), patch sizes [32, 64], Haar and BL5/3, float32 / binary16 / E4M3 records.
#include "lbmz_patch_kernel.h"

namespace lbmz {

bool dispatch_f32_euler(LBMZ_DISPATCH_ARGS) {
  if (k.dtype != 0 || k.scheme != S_EULER) return false;
  LBMZ_CASE_T(float, 32, W_HAAR, S_EULER, VF_F32)
  LBMZ_CASE_T(float, 32, W_BL53, S_EULER, VF_F32)
  LBMZ_CASE_T(float, 64, W_HAAR, S_EULER, VF_F32)
  LBMZ_CASE_T(float, 64, W_BL53, S_EULER, VF_F32)
  LBMZ_CASE_T(float, 32, W_HAAR, S_EULER, VF_F16)
  LBMZ_CASE_T(float, 32, W_BL53, S_EULER, VF_F16)
  LBMZ_CASE_T(float, 64, W_HAAR, S_EULER, VF_F16)
  LBMZ_CASE_T(float, 64, W_BL53, S_EULER, VF_F16)
  LBMZ_CASE_T(float, 32, W_HAAR, S_EULER, VF_E4M3)
  LBMZ_CASE_T(float, 32, W_BL53, S_EULER, VF_E4M3)
  LBMZ_CASE_T(float, 64, W_HAAR, S_EULER, VF_E4M3)
  LBMZ_CASE_T(float, 64, W_BL53, S_EULER, VF_E4M3)
  return false;
}

}  // namespace lbmz
