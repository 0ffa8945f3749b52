// Kernel instantiations: float, scheme S_LBM, bounded E4M3 records (E4M3 or binary16 details per record).
#include "lbmz_patch_kernel.h"

namespace lbmz {

bool dispatch_f32_e4m3b_lbm(LBMZ_DISPATCH_ARGS) {
  if (k.dtype != 0 || k.scheme != S_LBM || k.vf != VF_E4M3B) return false;
  LBMZ_CASE_T(float, 32, W_BL53, S_LBM, VF_E4M3B)
  LBMZ_CASE_T(float, 64, W_HAAR, S_LBM, VF_E4M3B)
  LBMZ_CASE_T(float, 64, W_BL53, S_LBM, VF_E4M3B)
  return false;
}

}  // namespace lbmz
