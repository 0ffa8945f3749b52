// Kernel instantiations: float, scheme S_LBM, patch sizes [32, 64], Haar and BL5/3, narrow records (binary16 and E4M3 details).
#include "lbmz_patch_kernel.h"

namespace lbmz {

bool dispatch_f32_lbm_q(LBMZ_DISPATCH_ARGS) {
  if (k.dtype != 0 || k.scheme != S_LBM) return false;
  LBMZ_CASE_T(float, 32, W_HAAR, S_LBM, VF_F16)
  LBMZ_CASE_T(float, 32, W_BL53, S_LBM, VF_F16)
  LBMZ_CASE_T(float, 64, W_HAAR, S_LBM, VF_F16)
  LBMZ_CASE_T(float, 64, W_BL53, S_LBM, VF_F16)
  LBMZ_CASE_T(float, 32, W_HAAR, S_LBM, VF_E4M3)
  LBMZ_CASE_T(float, 32, W_BL53, S_LBM, VF_E4M3)
  LBMZ_CASE_T(float, 64, W_HAAR, S_LBM, VF_E4M3)
  LBMZ_CASE_T(float, 64, W_BL53, S_LBM, VF_E4M3)
  return false;
}

}  // namespace lbmz
