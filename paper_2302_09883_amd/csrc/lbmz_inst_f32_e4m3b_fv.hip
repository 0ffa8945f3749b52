// Kernel instantiations: float, schemes S_FV and S_EULER, bounded E4M3 records (E4M3 or binary16 details per record).
#include "lbmz_patch_kernel.h"

namespace lbmz {

bool dispatch_f32_e4m3b_fv(LBMZ_DISPATCH_ARGS) {
  if (k.dtype != 0 || k.vf != VF_E4M3B) return false;
  if (k.scheme == S_FV) {
    LBMZ_CASE_T(float, 32, W_HAAR, S_FV, VF_E4M3B)
    LBMZ_CASE_T(float, 64, W_BL53, S_FV, VF_E4M3B)
  } else if (k.scheme == S_EULER) {
    LBMZ_CASE_T(float, 64, W_HAAR, S_EULER, VF_E4M3B)
    LBMZ_CASE_T(float, 64, W_BL53, S_EULER, VF_E4M3B)
  }
  return false;
}

}  // namespace lbmz
