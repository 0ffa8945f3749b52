// Kernel instantiations: double, scheme S_LBM (D2Q9 BGK), patch sizes [8, 16, 32], Haar and BL5/3, double records.
#include "lbmz_patch_kernel.h"

namespace lbmz {

bool dispatch_f64_lbm(LBMZ_DISPATCH_ARGS) {
  if (k.dtype != 1 || k.scheme != S_LBM) return false;
  LBMZ_CASE_T(double, 8, W_HAAR, S_LBM, VF_F32)
  LBMZ_CASE_T(double, 8, W_BL53, S_LBM, VF_F32)
  LBMZ_CASE_T(double, 16, W_HAAR, S_LBM, VF_F32)
  LBMZ_CASE_T(double, 16, W_BL53, S_LBM, VF_F32)
  LBMZ_CASE_T(double, 32, W_HAAR, S_LBM, VF_F32)
  LBMZ_CASE_T(double, 32, W_BL53, S_LBM, VF_F32)
  return false;
}

}  // namespace lbmz
